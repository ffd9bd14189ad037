// Host side of the C ABI declared in include/jet.h: argument checks, device memory, the Jet loop of
// Algorithm 1 (temperature rounds, locking, rollback), the rebalancing rounds of Section 4.3, and
// the inspection entry points.  All arithmetic on the partition runs in the HIP kernels; the host
// only launches them and reads back a small status block between phases.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "jet_internal.h"
#include "phi.h"

using jet::Ctx;
using jet::DevStatus;

struct jet_ctx {
  Ctx c;
};


namespace {

thread_local std::string g_init_error;

int fail(Ctx *c, int code, const std::string &msg) {
  if (c) c->last_error = msg;
  else g_init_error = msg;
  return code;
}

int fail_hip(Ctx *c, hipError_t e, const char *what) {
  return fail(c, JET_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_OR_FAIL(c, expr)                          \
  do {                                                \
    hipError_t _e = (expr);                           \
    if (_e != hipSuccess) return fail_hip(c, _e, #expr); \
  } while (0)

template <typename T>
hipError_t dalloc(T **p, size_t count) {
  *p = nullptr;  // stays null if the allocation fails
  return hipMalloc((void **)p, sizeof(T) * (count ? count : 1));
}

// status fields the loop needs each phase: counters, then the block weights of every segment (the
// rebalancing scratch after them is not copied)
// segments of a context: its blocks, or (union) the blocks of every hypergraph and of the padding
int64_t segments(const Ctx &c) { return (c.H > 1 ? (int64_t)c.H + 1 : 1) * c.k; }
size_t status_bytes(const Ctx &c) { return offsetof(DevStatus, bw) + sizeof(int64_t) * (size_t)segments(c); }

int map_device_error(Ctx &c, int32_t err, int32_t arg) {
  switch (err) {
  case jet::kErrPartRange: return fail(&c, JET_EINVAL, "part[" + std::to_string(arg) + "] outside [0,k)");
  case jet::kErrPinRange: return fail(&c, JET_EINVAL, "pin at index " + std::to_string(arg) + " outside [0,n)");
  case jet::kErrDupPin: return fail(&c, JET_EINVAL, "vertex " + std::to_string(arg) + " appears twice in one net");
  case jet::kErrDegree:
    return fail(&c, JET_EUNSUPPORTED,
                "vertex " + std::to_string(arg) + " has more than " + std::to_string(jet::kMaxSortedDegree) +
                    " incident nets");
  case jet::kErrMixedOverflow:
    return fail(&c, JET_EUNSUPPORTED,
                "net " + std::to_string(arg) + ": more than " + std::to_string(jet::kBigCap) +
                    " ordered afterburner events on blocks that every pin leaves");
  case jet::kErrWeight: return fail(&c, JET_EINVAL, "a vertex or net weight is below 1");
  case jet::kErrTarget:
    return fail(&c, JET_EINVAL, "candidate " + std::to_string(arg) + " has a target outside [0,k) or equal to its block");
  case jet::kErrOverflow:
    return fail(&c, JET_EOVERFLOW, "incident net weight of vertex " + std::to_string(arg) + " reaches 2^31");
  default: return fail(&c, JET_EINVAL, "device reported error " + std::to_string(err));
  }
}

int read_status(Ctx &c) {
  HIP_OR_FAIL(&c, hipMemcpyAsync(c.hst, c.st, status_bytes(c), hipMemcpyDeviceToHost, c.stream));
  HIP_OR_FAIL(&c, hipStreamSynchronize(c.stream));
  for (int i = 0; i < jet::kKm1Slots; ++i) c.hst->km1 += c.hst->km1_slot[i];  // the metric (host view)
  if (c.hst->err != 0) {
    const int32_t err = c.hst->err, arg = c.hst->err_arg;
    (void)hipMemsetAsync(&c.st->err, 0, 2 * sizeof(int32_t), c.stream);
    (void)hipStreamSynchronize(c.stream);
    return map_device_error(c, err, arg);
  }
  return JET_OK;
}

int64_t overload(const Ctx &c) {
  int64_t worst = 0;
  for (int b = 0; b < c.k; ++b) worst = std::max(worst, c.hst->bw[b] - c.lmax);
  return worst;
}

int64_t max_block_weight(const Ctx &c) {
  int64_t mx = 0;
  for (int b = 0; b < c.k; ++b) mx = std::max(mx, c.hst->bw[b]);
  return mx;
}

// Balance limit and deadzone (Section 2, Section 4.3) as integer thresholds, in IEEE double:
//   Lmax = floor((1+eps) A), DZ = ceil((1+eps) A - d eps A), A = ceil(W/k).
void limits(int64_t W, int32_t k, double eps, int32_t deadzone_ppm, int64_t *A, int64_t *lmax, int64_t *dz) {
  const int64_t a = (W + k - 1) / k;
  const double ad = (double)a;
  const double lreal = (1.0 + eps) * ad;
  const double dreal = lreal - ((double)deadzone_ppm / 1e6) * eps * ad;
  *A = a;
  *lmax = (int64_t)std::floor(lreal);
  *dz = (int64_t)std::ceil(dreal);
}

int32_t quantize_tau(float tau) { return (int32_t)std::floor((double)tau * 65536.0 + 0.5); }

int check_params(Ctx &c, const jet_params *p, bool loop) {
  if (!p) return fail(&c, JET_EINVAL, "params is NULL");
  if (p->deadzone_ppm < 0 || p->deadzone_ppm > 1000000) return fail(&c, JET_EINVAL, "deadzone_ppm outside [0,1e6]");
  if (p->max_rebalance_rounds < 0) return fail(&c, JET_EINVAL, "max_rebalance_rounds < 0");
  if (p->rb_unweighted < 0 || p->rb_unweighted > 2) return fail(&c, JET_EINVAL, "rb_unweighted must be 0, 1 or 2");
  if (!loop) return JET_OK;
  if (p->limit < 1 || p->max_iters < 1) return fail(&c, JET_EINVAL, "limit and max_iters must be >= 1");
  if (p->num_tau < 1 || p->num_tau > 8) return fail(&c, JET_EINVAL, "num_tau outside [1,8]");
  for (int r = 0; r < p->num_tau; ++r)
    if (!(p->tau[r] >= 0.0f && p->tau[r] <= 1.0f)) return fail(&c, JET_EINVAL, "tau outside [0,1]");
  return JET_OK;
}

// Builds pin counts, connectivity words, block weights and the metric from part.
int build_state(Ctx &c, const int32_t *part) {
  if (!part) return fail(&c, JET_EINVAL, "part is NULL");
  HIP_OR_FAIL(&c, jet::launch_check_part(c, part));
  int rc = read_status(c);
  if (rc != JET_OK) return rc;
  HIP_OR_FAIL(&c, c.phi16 ? jet::launch_build_phi(c, part, c.phi16) : jet::launch_build_phi(c, part, c.phi));
  HIP_OR_FAIL(&c, jet::launch_build_ns(c));
  HIP_OR_FAIL(&c, jet::launch_block_weights(c, part));
  HIP_OR_FAIL(&c, jet::launch_km1_from_ns(c));
  return read_status(c);
}

// Moves the listed vertices and keeps every derived structure consistent.
// kind 0: Jet moves, 1: rebalancing moves, 2: anything else (no hint kept)
int apply_and_read(Ctx &c, int32_t *part, int kind) {
  HIP_OR_FAIL(&c, jet::launch_apply_moves(c, part, c.wide_enabled && kind < 2 && c.wide_hint[kind]));
  const int rc = read_status(c);
  if (rc == JET_OK && kind < 2)
    c.wide_hint[kind] = c.apply_divisor > 0 && c.hst->mv_inc * c.apply_divisor >= c.p;
  return rc;
}

void final_stats(const Ctx &c, jet_stats *st) {
  st->km1_out = c.hst->km1;
  st->lmax = c.lmax;
  st->max_block_weight = max_block_weight(c);
  st->balanced = st->max_block_weight <= c.lmax;
}

void drop_graph(Ctx &c);

// The clustering state (allocated at the first clustering call).
void co_free(Ctx &c) {
  if (!c.co) return;
  jet::CoState &s = *c.co;
  for (void *p : {(void *)s.qnet, (void *)s.deg, (void *)s.cw, (void *)s.tp, (void *)s.tt, (void *)s.gcnt,
                  (void *)s.gslot, (void *)s.newlab, (void *)s.flag, (void *)s.jw, (void *)s.gpos,
                  (void *)s.gtarget, (void *)s.members, (void *)s.goff, (void *)s.gmoved, (void *)s.ptab,
                  (void *)s.tab, (void *)s.ctr})
    if (p) (void)hipFree(p);
  delete c.co;
  c.co = nullptr;
}

void free_ctx(Ctx &c) {
  void *ptrs[] = {c.off,  c.pins, c.nw,   c.vw,        c.voff, c.inc,   c.sumw, c.adj,    c.chunks,    c.pnet, c.mid_nets,
                  c.big_nets, c.phi, c.phi16, c.ns, c.rec, c.inm, c.rg, c.lockstamp, c.best, c.moves, c.rb_keys,
                  c.rb_target, c.st, c.scan_tmp, c.ovf_list, c.ovf_off, c.ovf_ka, c.ovf_kb, c.ovf_ma,
                  c.ovf_mb, c.hubs, c.mvto, c.bigmv, c.rb_list, c.rb_slot, c.lstat, c.tau_io, c.rgx, c.rb_hlist, c.rb_hacc,
                  c.rb_keys2, c.rb_gw, c.rb_gc};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  if (c.hst) (void)hipHostFree(c.hst);
  drop_graph(c);
  if (c.gstream) (void)hipStreamDestroy(c.gstream);
  for (void *p : {(void *)c.lc, (void *)c.cpart, (void *)c.dtrace, (void *)c.dprof, (void *)c.vhg, (void *)c.nhg,
                  (void *)c.act, (void *)c.ht0, (void *)c.hch0})
    if (p) (void)hipFree(p);
  if (c.lcs && c.lcs != c.lc) (void)hipFree(c.lcs);
  co_free(c);
  jet::flow_free(c);
  if (c.hlc) (void)hipHostFree(c.hlc);
  if (c.hlcs && c.hlcs != c.hlc) (void)hipHostFree(c.hlcs);
}

int init_impl(Ctx &c, int32_t n, int32_t m, int64_t num_pins, const int64_t *net_offsets, const int32_t *pins,
              const int32_t *net_weights, const int32_t *vertex_weights) {
  c.n = n;
  c.m = m;
  c.p = num_pins;
  c.nw_words = c.k > 64 ? 2 : 1;
  c.unit_nw = net_weights == nullptr;
  c.unit_vw = vertex_weights == nullptr;
  if (const char *env = std::getenv("JET_APPLY_DIVISOR")) c.apply_divisor = std::max(0, std::atoi(env));
  if (const char *env = std::getenv("JET_APPLY_WIDE")) c.wide_enabled = std::atoi(env) != 0;
  if (const char *env = std::getenv("JET_CAND_LANE_DEGREE")) c.lane_degree = std::max(0, std::atoi(env));
  if (const char *env = std::getenv("JET_CAND_XCD")) c.cand_xcd = std::atoi(env) != 0;
  if (const char *env = std::getenv("JET_RB_XCD")) c.rb_xcd = std::atoi(env) != 0;
  if (const char *env = std::getenv("JET_GRAPH_KERNELS")) c.graph_kernels = std::atoi(env) != 0;
  if (const char *env = std::getenv("JET_APPLY_XCD")) c.apply_xcd = std::atoi(env) != 0;
  if (const char *env = std::getenv("JET_SEL_SPLIT_MIN")) c.sel_split_min = std::max(0, std::atoi(env));
  if (const char *env = std::getenv("JET_SEL_SLICES")) c.sel_slices = std::max(0, std::min(64, std::atoi(env)));
  HIP_OR_FAIL(&c, hipHostMalloc((void **)&c.hst, sizeof(DevStatus)));
  HIP_OR_FAIL(&c, dalloc(&c.st, 1));
  HIP_OR_FAIL(&c, hipMemsetAsync(c.st, 0, sizeof(DevStatus), c.stream));
  HIP_OR_FAIL(&c, dalloc(&c.off, (size_t)m + 1));
  HIP_OR_FAIL(&c, dalloc(&c.pins, (size_t)num_pins));
  HIP_OR_FAIL(&c, hipMemcpyAsync(c.off, net_offsets, sizeof(int64_t) * ((size_t)m + 1), hipMemcpyDefault, c.stream));
  HIP_OR_FAIL(&c, hipMemcpyAsync(c.pins, pins, sizeof(int32_t) * (size_t)num_pins, hipMemcpyDefault, c.stream));
  if (net_weights) {
    HIP_OR_FAIL(&c, dalloc(&c.nw, (size_t)m));
    HIP_OR_FAIL(&c, hipMemcpyAsync(c.nw, net_weights, sizeof(int32_t) * (size_t)m, hipMemcpyDefault, c.stream));
  }
  if (vertex_weights) {
    HIP_OR_FAIL(&c, dalloc(&c.vw, (size_t)n));
    HIP_OR_FAIL(&c, hipMemcpyAsync(c.vw, vertex_weights, sizeof(int32_t) * (size_t)n, hipMemcpyDefault, c.stream));
  }
  // offsets: validated and scheduled on the host
  std::vector<int64_t> hoff((size_t)m + 1);
  HIP_OR_FAIL(&c, hipMemcpyAsync(hoff.data(), c.off, sizeof(int64_t) * ((size_t)m + 1), hipMemcpyDeviceToHost,
                                  c.stream));
  HIP_OR_FAIL(&c, hipStreamSynchronize(c.stream));
  if (hoff[0] != 0 || hoff[m] != num_pins) return fail(&c, JET_EINVAL, "net_offsets must start at 0 and end at num_pins");
  for (int32_t e = 0; e < m; ++e)
    if (hoff[e + 1] <= hoff[e]) return fail(&c, JET_EINVAL, "net " + std::to_string(e) + " is empty or offsets decrease");
  // weights and total vertex weight
  HIP_OR_FAIL(&c, jet::launch_check_weights(c));
  int rc = read_status(c);
  if (rc != JET_OK) return rc;
  c.W = vertex_weights ? c.hst->bw[0] : (int64_t)n;
  // a union checks each of its hypergraphs' totals instead (done before this call)
  if (c.H == 1 && c.W > INT32_MAX) return fail(&c, JET_EOVERFLOW, "total vertex weight reaches 2^31");
  int64_t dz_unused;
  limits(c.W, c.k, c.eps, 0, &c.A, &c.lmax, &dz_unused);
  // incidence lists I(v)
  HIP_OR_FAIL(&c, dalloc(&c.voff, (size_t)n + 1));
  HIP_OR_FAIL(&c, dalloc(&c.inc, (size_t)num_pins));
  HIP_OR_FAIL(&c, dalloc(&c.sumw, (size_t)n));
  {
    int32_t *deg = nullptr;
    HIP_OR_FAIL(&c, dalloc(&deg, (size_t)n));
    hipError_t e = hipMemsetAsync(deg, 0, sizeof(int32_t) * (size_t)n, c.stream);
    if (e == hipSuccess) e = jet::launch_degrees(c, deg);
    if (e == hipSuccess) e = jet::launch_exclusive_scan_i32_to_i64(c, deg, c.voff, n);
    if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
    (void)hipFree(deg);
    if (e != hipSuccess) return fail_hip(&c, e, "incidence degrees");
  }
  rc = read_status(c);
  if (rc != JET_OK) return rc;
  {
    int64_t *cursor = nullptr;
    HIP_OR_FAIL(&c, dalloc(&cursor, (size_t)n));
    hipError_t e = hipMemcpyAsync(cursor, c.voff, sizeof(int64_t) * (size_t)n, hipMemcpyDeviceToDevice, c.stream);
    if (e == hipSuccess) e = jet::launch_fill_incidence(c, cursor);
    if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
    (void)hipFree(cursor);
    if (e != hipSuccess) return fail_hip(&c, e, "incidence fill");
  }
  HIP_OR_FAIL(&c, jet::launch_sort_incidence(c));
  rc = read_status(c);
  if (rc != JET_OK) return rc;
  {  // hubs: vertices whose incident nets are split over a whole workgroup
    std::vector<int64_t> hvoff((size_t)n + 1);
    HIP_OR_FAIL(&c, hipMemcpyAsync(hvoff.data(), c.voff, sizeof(int64_t) * ((size_t)n + 1), hipMemcpyDeviceToHost,
                                    c.stream));
    HIP_OR_FAIL(&c, hipStreamSynchronize(c.stream));
    std::vector<int32_t> hh;
    c.n_low = 0;
    c.p_low = 0;
    for (int32_t v = 0; v < n; ++v) {
      const int64_t d = hvoff[v + 1] - hvoff[v];
      if (d > jet::kHubDegree) {
        hh.push_back(v);
      } else {
        c.n_low += 1;
        c.p_low += d;
      }
    }
    c.nhubs = (int32_t)hh.size();
    HIP_OR_FAIL(&c, dalloc(&c.hubs, hh.size()));
    HIP_OR_FAIL(&c, dalloc(&c.rb_hlist, hh.size()));
    HIP_OR_FAIL(&c, dalloc(&c.rb_hacc, hh.size() * (size_t)(c.k + 1)));
    HIP_OR_FAIL(&c, hipMemsetAsync(c.rb_hacc, 0, sizeof(int32_t) * hh.size() * (size_t)(c.k + 1), c.stream));
    if (!hh.empty())
      HIP_OR_FAIL(&c, hipMemcpyAsync(c.hubs, hh.data(), sizeof(int32_t) * hh.size(), hipMemcpyHostToDevice, c.stream));
  }
  // net schedule: chunks of consecutive small nets (<= 64 pins in total), medium and big net lists
  std::vector<int4> chunks;
  std::vector<std::pair<int64_t, int32_t>> mid, big;
  int32_t cur_first = -1, cur_cnt = 0;
  int64_t cur_pins = 0;
  auto close = [&]() {
    if (cur_cnt > 0)
      chunks.push_back(make_int4(cur_first, cur_cnt, (int32_t)cur_pins, (int32_t)hoff[cur_first]));
    cur_first = -1;
    cur_cnt = 0;
    cur_pins = 0;
  };
  std::vector<int32_t> hch0;  // union: first chunk of every hypergraph (no chunk spans two)
  size_t next_hg = 0;
  for (int32_t e = 0; e < m; ++e) {
    while (c.H > 1 && next_hg < (size_t)c.H && e == c.hg_e0[next_hg]) {
      close();
      hch0.push_back((int32_t)chunks.size());
      ++next_hg;
    }
    const int64_t sz = hoff[e + 1] - hoff[e];
    if (sz > jet::kSmallNet) {
      close();
      (sz > jet::kMediumNet ? big : mid).push_back({sz, e});
      continue;
    }
    if (cur_cnt > 0 && cur_pins + sz > jet::kSmallNet) close();
    if (cur_cnt == 0) cur_first = e;
    cur_cnt += 1;
    cur_pins += sz;
  }
  close();
  while (c.H > 1 && hch0.size() < (size_t)c.H + 1) hch0.push_back((int32_t)chunks.size());
  auto by_size = [](const std::pair<int64_t, int32_t> &a, const std::pair<int64_t, int32_t> &b) {
    return a.first != b.first ? a.first > b.first : a.second < b.second;
  };
  std::sort(mid.begin(), mid.end(), by_size);
  std::sort(big.begin(), big.end(), by_size);
  std::vector<int32_t> hmid(mid.size()), hbig(big.size());
  for (size_t i = 0; i < mid.size(); ++i) hmid[i] = mid[i].second;
  for (size_t i = 0; i < big.size(); ++i) hbig[i] = big[i].second;
  c.nchunks = (int32_t)chunks.size();
  c.nmid = (int32_t)hmid.size();
  c.nmid_large = 0;
  while (c.nmid_large < c.nmid && mid[c.nmid_large].first > jet::kMediumSmall) ++c.nmid_large;
  c.nbig = (int32_t)hbig.size();
  // nets that may need the global-scratch afterburner: more pins than the in-LDS capacity
  std::vector<int64_t> hovf(1, 0);
  for (const auto &b : big) {
    if (b.first <= jet::kBigCap) break;
    if (b.first >= (int64_t)1 << 30) return fail(&c, JET_EUNSUPPORTED, "a net has 2^30 or more pins");
    hovf.push_back(hovf.back() + 2 * b.first);
  }
  c.nbig_over = (int32_t)hovf.size() - 1;
  if (c.nbig_over > 0) {
    const size_t slots = (size_t)hovf.back();
    HIP_OR_FAIL(&c, dalloc(&c.ovf_list, (size_t)c.nbig_over));
    HIP_OR_FAIL(&c, dalloc(&c.ovf_off, hovf.size()));
    HIP_OR_FAIL(&c, hipMemcpyAsync(c.ovf_off, hovf.data(), sizeof(int64_t) * hovf.size(), hipMemcpyHostToDevice,
                                    c.stream));
    HIP_OR_FAIL(&c, dalloc(&c.ovf_ka, slots));
    HIP_OR_FAIL(&c, dalloc(&c.ovf_kb, slots));
    HIP_OR_FAIL(&c, dalloc(&c.ovf_ma, slots));
    HIP_OR_FAIL(&c, dalloc(&c.ovf_mb, slots));
  }
  HIP_OR_FAIL(&c, dalloc(&c.chunks, chunks.size()));
  {
    std::vector<uint8_t> hpnet((size_t)num_pins, 0xff);
    for (const int4 &cd : chunks)
      for (int32_t j = 0; j < cd.y; ++j)
        for (int64_t q = hoff[cd.x + j]; q < hoff[cd.x + j + 1]; ++q) hpnet[q] = (uint8_t)j;
    HIP_OR_FAIL(&c, dalloc(&c.pnet, (size_t)num_pins));
    HIP_OR_FAIL(&c, hipMemcpy(c.pnet, hpnet.data(), (size_t)num_pins, hipMemcpyHostToDevice));
  }
  HIP_OR_FAIL(&c, dalloc(&c.mid_nets, hmid.size()));
  HIP_OR_FAIL(&c, dalloc(&c.big_nets, hbig.size()));
  if (!chunks.empty())
    HIP_OR_FAIL(&c, hipMemcpyAsync(c.chunks, chunks.data(), sizeof(int4) * chunks.size(), hipMemcpyHostToDevice,
                                    c.stream));
  if (c.H > 1) {  // union: first tile and first chunk of every hypergraph, lists per phase
    std::vector<int32_t> ht0((size_t)c.H + 1);
    for (int32_t h = 0; h <= c.H; ++h) ht0[h] = c.hg_v0[h] / jet::kUnionTile;
    HIP_OR_FAIL(&c, dalloc(&c.ht0, ht0.size()));
    HIP_OR_FAIL(&c, dalloc(&c.hch0, hch0.size()));
    HIP_OR_FAIL(&c, hipMemcpy(c.ht0, ht0.data(), sizeof(int32_t) * ht0.size(), hipMemcpyHostToDevice));
    HIP_OR_FAIL(&c, hipMemcpy(c.hch0, hch0.data(), sizeof(int32_t) * hch0.size(), hipMemcpyHostToDevice));
    HIP_OR_FAIL(&c, dalloc(&c.act, jet::kActLists));
    HIP_OR_FAIL(&c, hipMemset(c.act, 0, sizeof(jet::ActList) * jet::kActLists));
  }
  if (!hmid.empty())
    HIP_OR_FAIL(&c, hipMemcpyAsync(c.mid_nets, hmid.data(), sizeof(int32_t) * hmid.size(), hipMemcpyHostToDevice,
                                    c.stream));
  if (!hbig.empty())
    HIP_OR_FAIL(&c, hipMemcpyAsync(c.big_nets, hbig.data(), sizeof(int32_t) * hbig.size(), hipMemcpyHostToDevice,
                                    c.stream));
  // partition state
  {
    int64_t maxsz = 0;
    for (int32_t e = 0; e < m; ++e) maxsz = std::max<int64_t>(maxsz, hoff[e + 1] - hoff[e]);
    if (maxsz <= 65535) HIP_OR_FAIL(&c, dalloc(&c.phi16, jet::phi_entries(m, c.k)));
    else HIP_OR_FAIL(&c, dalloc(&c.phi, jet::phi_entries(m, c.k)));
    if (maxsz == 2 && num_pins == 2 * (int64_t)m) {  // a graph: every net has two pins
      HIP_OR_FAIL(&c, dalloc(&c.adj, (size_t)num_pins));
      HIP_OR_FAIL(&c, jet::launch_build_adj(c));
    }
  }
  HIP_OR_FAIL(&c, dalloc(&c.ns, (size_t)m * 2 * c.nw_words));
  HIP_OR_FAIL(&c, dalloc(&c.rec, (size_t)n));
  const size_t inm_words = ((size_t)n + 255) / 256 * 8;
  HIP_OR_FAIL(&c, dalloc(&c.inm, inm_words));
  HIP_OR_FAIL(&c, hipMemsetAsync(c.inm, 0, sizeof(uint32_t) * inm_words, c.stream));
  HIP_OR_FAIL(&c, dalloc(&c.rg, (size_t)n));
  // small levels of heavy vertices (a few hot counters): 64 private copies of the recomputed gains
  // for the afterburner (at most 16 MB); with light vertices the atomics rarely collide and the
  // copies would only add their summing pass
  c.rg_copies = n <= 65536 && num_pins >= 256 * (int64_t)n ? 64 : 1;
  if (c.rg_copies > 1) {
    HIP_OR_FAIL(&c, dalloc(&c.rgx, (size_t)c.rg_copies * n));
    HIP_OR_FAIL(&c, hipMemsetAsync(c.rgx, 0, sizeof(int32_t) * (size_t)c.rg_copies * n, c.stream));
  }
  HIP_OR_FAIL(&c, hipMemsetAsync(c.rg, 0, sizeof(int32_t) * (size_t)n, c.stream));
  HIP_OR_FAIL(&c, dalloc(&c.lockstamp, (size_t)n));
  HIP_OR_FAIL(&c, hipMemsetAsync(c.lockstamp, 0x80, sizeof(int32_t) * (size_t)n, c.stream));  // never moved
  HIP_OR_FAIL(&c, dalloc(&c.best, (size_t)n));
  HIP_OR_FAIL(&c, dalloc(&c.moves, (size_t)n));
  HIP_OR_FAIL(&c, dalloc(&c.mvto, (size_t)n));
  HIP_OR_FAIL(&c, dalloc(&c.bigmv, (size_t)n));
  HIP_OR_FAIL(&c, dalloc(&c.rb_list, (size_t)n));
  HIP_OR_FAIL(&c, dalloc(&c.rb_slot, (size_t)n));
  HIP_OR_FAIL(&c, dalloc(&c.lstat, 5));
  HIP_OR_FAIL(&c, dalloc(&c.tau_io, 17));
  HIP_OR_FAIL(&c, hipMemsetAsync(c.mvto, 0xff, (size_t)n, c.stream));
  HIP_OR_FAIL(&c, dalloc(&c.rb_keys, (size_t)n * 8));
  HIP_OR_FAIL(&c, dalloc(&c.rb_keys2, (size_t)n * 8));
  HIP_OR_FAIL(&c, dalloc(&c.rb_gw, (size_t)jet::kMaxK * 256));
  HIP_OR_FAIL(&c, dalloc(&c.rb_gc, (size_t)jet::kMaxK * 256));
  HIP_OR_FAIL(&c, hipMemsetAsync(c.rb_gw, 0, sizeof(unsigned long long) * jet::kMaxK * 256, c.stream));
  HIP_OR_FAIL(&c, hipMemsetAsync(c.rb_gc, 0, sizeof(uint32_t) * jet::kMaxK * 256, c.stream));
  // device-resident loop: record, working partition, iteration records, timing accumulators
  HIP_OR_FAIL(&c, dalloc(&c.lc, 1));
  HIP_OR_FAIL(&c, hipMemsetAsync(c.lc, 0, sizeof(jet::LoopCtl), c.stream));
  HIP_OR_FAIL(&c, hipHostMalloc((void **)&c.hlc, sizeof(jet::LoopCtl)));
  std::memset(c.hlc, 0, sizeof(jet::LoopCtl));
  if (c.H == 1) {  // the record is the gate record (a union gets per-hypergraph records on top)
    c.lcs = c.lc;
    c.hlcs = c.hlc;
  }
  HIP_OR_FAIL(&c, dalloc(&c.cpart, (size_t)n));
  c.dtrace_cap = 4096;
  HIP_OR_FAIL(&c, dalloc(&c.dtrace, (size_t)c.dtrace_cap));
  HIP_OR_FAIL(&c, dalloc(&c.dprof, 1));
  HIP_OR_FAIL(&c, hipMemsetAsync(c.dprof, 0, sizeof(jet::DevProf), c.stream));
  HIP_OR_FAIL(&c, hipStreamCreateWithFlags(&c.gstream, hipStreamNonBlocking));
  {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
      c.wall_khz = (double)khz;
  }
  if (const char *env = std::getenv("JET_GRAPH")) c.use_graph = std::atoi(env) != 0;
  HIP_OR_FAIL(&c, hipStreamSynchronize(c.stream));
  return JET_OK;
}

// A call's parameters in a hypergraph's loop record (the device completes it); the stamp continues
// from the record's last value, so lock stamps of earlier calls never match.
void fill_record(jet::LoopCtl &r, const jet_params &prm, bool rb_only, int32_t trace_cap, int64_t lmax, int64_t dz,
                 int64_t A) {
  const int32_t stamp = r.stamp;
  std::memset(&r, 0, sizeof r);
  r.stamp = stamp + 2;  // nothing was moved in the iteration before the first one: no locks
  r.limit = prm.limit;
  r.max_iters = prm.max_iters;
  r.num_tau = rb_only ? 1 : prm.num_tau;
  r.max_rb = prm.max_rebalance_rounds;
  for (int i = 0; i < 8; ++i) r.tau_qs[i] = (!rb_only && i < prm.num_tau) ? quantize_tau(prm.tau[i]) : 0;
  r.tau_q = r.tau_qs[0];
  r.rb_only = rb_only ? 1 : 0;
  r.rb_unw = prm.rb_unweighted;
  r.trace_cap = trace_cap;
  r.lmax = lmax;
  r.dz = dz;
  r.A = A;
  r.phase = rb_only ? jet::kPhRb : jet::kPhJet;
  r.phase_mask = 1 << r.phase;
}

void drop_graph(Ctx &c) {
  for (int i = 0; i < 4; ++i) {
    if (c.gexec[i]) (void)hipGraphExecDestroy(c.gexec[i]);
    if (c.graph[i]) (void)hipGraphDestroy(c.graph[i]);
    c.gexec[i] = nullptr;
    c.graph[i] = nullptr;
  }
}

// The pieces of an iteration captured as graphs on the context's capture stream (once; dropped
// when an option or the instrumentation changes what they launch).
int ensure_graphs(Ctx &c) {
  if (c.gexec[0]) return JET_OK;
  for (int kind = 0; kind < 4; ++kind) {
    hipStream_t user = c.stream;
    c.stream = c.gstream;
    hipError_t e = hipStreamBeginCapture(c.gstream, hipStreamCaptureModeThreadLocal);
    hipError_t le = hipSuccess;
    if (e == hipSuccess) {
      le = jet::launch_tick(c, kind);
      e = hipStreamEndCapture(c.gstream, &c.graph[kind]);
    }
    c.stream = user;
    if (e == hipSuccess && le == hipSuccess) e = hipGraphInstantiate(&c.gexec[kind], c.graph[kind], nullptr, nullptr, 0);
    if (e != hipSuccess || le != hipSuccess) {
      drop_graph(c);
      return fail_hip(&c, e != hipSuccess ? e : le, "capturing the iteration graphs");
    }
  }
  return JET_OK;
}

int launch_piece(Ctx &c, int kind) {
  if (c.use_graph) HIP_OR_FAIL(&c, hipGraphLaunch(c.gexec[kind], c.stream));
  else HIP_OR_FAIL(&c, jet::launch_tick(c, kind));
  return JET_OK;
}

// The Jet loop (Algorithm 1) for every temperature, or (rb_only) the rebalancing rounds alone, on
// the device.  The host launches pieces of iterations and looks at the loop record between
// batches of them; what it launches only decides how much work is in flight, never what is
// computed: a piece whose phase the record is not in does nothing.
//   phase Jet: min(limit - round, max_iters - it) iterations at least remain in the round (fewer
//              only at a fixed point), up to `replays` of them are launched, each a Jet piece, or
//              a Jet + rebalancing piece once this call has seen a rebalancing round;
//   phase Rb:  rebalancing pieces, as many as the call's rounds per iteration so far suggest;
//   phase Roll: the rollback piece (the next round starts at the next look).
int run_loop(Ctx &c, int32_t *part, const jet_params *prm, bool rb_only, jet_stats *out, jet_trace *trace,
             int32_t trace_cap, int32_t *trace_len) {
  int rc = check_params(c, prm, !rb_only);
  if (rc != JET_OK) return rc;
  if (!part) return fail(&c, JET_EINVAL, "part is NULL");
  if (trace_cap < 0) trace_cap = 0;
  if (!trace) trace_cap = 0;
  int64_t A, lmax, dz;
  limits(c.W, c.k, c.eps, prm->deadzone_ppm, &A, &lmax, &dz);
  if (trace_cap > c.dtrace_cap) {
    drop_graph(c);  // the graphs hold the record array's address
    if (c.dtrace) (void)hipFree(c.dtrace);
    c.dtrace = nullptr;
    c.dtrace_cap = 0;
    HIP_OR_FAIL(&c, dalloc(&c.dtrace, (size_t)trace_cap));
    c.dtrace_cap = trace_cap;
  }
  HIP_OR_FAIL(&c, hipMemcpyAsync(c.cpart, part, sizeof(int32_t) * (size_t)c.n, hipMemcpyDeviceToDevice, c.stream));
  rc = build_state(c, c.cpart);
  if (rc != JET_OK) return rc;
  fill_record(c.hlcs[0], *prm, rb_only, trace_cap, c.lmax, dz, c.A);
  HIP_OR_FAIL(&c, hipMemcpyAsync(c.lcs, c.hlcs, sizeof(jet::LoopCtl), hipMemcpyHostToDevice, c.stream));
  HIP_OR_FAIL(&c, jet::launch_loop_init(c));
  if (!rb_only)
    HIP_OR_FAIL(&c, hipMemcpyAsync(c.best, c.cpart, sizeof(int32_t) * (size_t)c.n, hipMemcpyDeviceToDevice, c.stream));
  if (c.use_graph) {
    rc = ensure_graphs(c);
    if (rc != JET_OK) return rc;
  }
  const int64_t piece_cap = (int64_t)(rb_only ? 1 : prm->num_tau) * ((int64_t)prm->max_iters + 2) *
                                ((int64_t)prm->max_rebalance_rounds / std::max(1, c.rb_slots) + 3) + 16;
  int64_t pieces = 0;
  c.polls = 0;
  int32_t phase = rb_only ? jet::kPhRb : jet::kPhJet;
  int32_t left = 1, rb_left = 1;
  bool rb_seen = false;
  for (;;) {
    if (phase == jet::kPhRoll) {
      rc = launch_piece(c, jet::kTickRoll);
      pieces += 1;
    } else if (phase == jet::kPhRb) {
      for (int32_t g = 0; g < rb_left && rc == JET_OK; ++g) rc = launch_piece(c, jet::kTickRb);
      pieces += rb_left;
    } else {
      const int kind = rb_seen ? jet::kTickJetRb : jet::kTickJet;
      for (int32_t g = 0; g < left && rc == JET_OK; ++g) rc = launch_piece(c, kind);
      pieces += left;
    }
    if (rc != JET_OK) return rc;
    HIP_OR_FAIL(&c, hipMemcpyAsync(c.hlc, c.lc, sizeof(jet::LoopCtl), hipMemcpyDeviceToHost, c.stream));
    rc = read_status(c);
    c.polls += 1;
    if (rc != JET_OK) return rc;
    const jet::LoopCtl &h = *c.hlc;
    phase = h.phase;
    if (phase == jet::kPhDone) break;
    if (pieces > piece_cap) return fail(&c, JET_EHIP, "the device loop did not finish within its bound");
    rb_seen = rb_seen || h.rebalance_rounds > 0 || h.rb_rounds > 0;
    left = 1;
    if (phase == jet::kPhJet)
      left = (int32_t)std::max<int64_t>(1, std::min<int64_t>({(int64_t)h.limit - h.round,
                                                              (int64_t)h.max_iters - h.it, (int64_t)c.replays}));
    // rounds per iteration so far, less the rounds this iteration already ran, in pieces
    const int64_t per_it = h.iterations > 0 ? (h.rebalance_rounds + h.iterations - 1) / h.iterations : 1;
    const int64_t want = std::max<int64_t>(1, per_it - h.rb_rounds);
    rb_left = (int32_t)std::max<int64_t>(1, std::min<int64_t>((want + c.rb_slots - 1) / c.rb_slots, c.replays));
  }
  c.replays_done = pieces;
  HIP_OR_FAIL(&c, hipMemcpyAsync(part, c.cpart, sizeof(int32_t) * (size_t)c.n, hipMemcpyDeviceToDevice, c.stream));
  const jet::LoopCtl &h = *c.hlc;
  const int32_t ntrace = std::min(h.ntrace, trace_cap);
  if (ntrace > 0)
    HIP_OR_FAIL(&c, hipMemcpyAsync(trace, c.dtrace, sizeof(jet_trace) * (size_t)ntrace, hipMemcpyDeviceToHost,
                                   c.stream));
  HIP_OR_FAIL(&c, hipStreamSynchronize(c.stream));
  jet_stats S;
  std::memset(&S, 0, sizeof S);
  S.km1_in = h.km1_in;
  S.iterations = h.iterations;
  S.rebalance_rounds = h.rebalance_rounds;
  S.moves_executed = h.moves_executed;
  if (!rb_only)
    for (int r = 0; r < prm->num_tau; ++r) S.tau_q_used[r] = quantize_tau(prm->tau[r]);
  final_stats(c, &S);
  S.km1_out = h.km1;
  if (out) *out = S;
  if (trace_len) *trace_len = h.ntrace;
  return S.balanced ? JET_OK : JET_IMBALANCED;
}

int refine_impl(Ctx &c, int32_t *part, const jet_params *prm, jet_stats *out, jet_trace *trace, int32_t trace_cap,
                int32_t *trace_len) {
  return run_loop(c, part, prm, false, out, trace, trace_cap, trace_len);
}


// ---- synchronous clustering (Section 6, Algorithm 4): host side ----

// rating-table slots of a vertex with d = sum of (|e| - 1) over its nets: a power of two at least
// twice the number of clusters it can meet (at most min(d, n)), so probing stays short
int64_t co_table(int64_t d, int64_t n) {
  if (d <= 0) return 0;
  const int64_t want = std::max<int64_t>(16, 2 * std::min(d, n));
  int64_t t = 16;
  while (t < want) t <<= 1;
  return t;
}

// (first position, length) of every sub-round: initial_single of one vertex, then 2, 4, 8, ... up
// to max(1, n / cap_div) (Section 6, prefix doubling)
std::vector<std::pair<int64_t, int64_t>> co_schedule(int64_t n, int32_t initial_single, int32_t cap_div) {
  std::vector<std::pair<int64_t, int64_t>> r;
  const int64_t cap = std::max<int64_t>(1, n / cap_div);
  int64_t s = 0, len = 1;
  for (int64_t i = 0; s < n; ++i) {
    if (i < initial_single) len = 1;
    else if (i == initial_single) len = std::min<int64_t>(2, cap);
    else len = std::min<int64_t>(2 * len, cap);
    const int64_t l = std::min(len, n - s);
    r.emplace_back(s, l);
    s += l;
  }
  return r;
}

int co_alloc(Ctx &c) {
  jet::CoState &s = *c.co;
  const size_t n = (size_t)c.n;
  HIP_OR_FAIL(&c, dalloc(&s.qnet, (size_t)c.m));
  HIP_OR_FAIL(&c, dalloc(&s.deg, n));
  HIP_OR_FAIL(&c, dalloc(&s.cw, n));
  for (int32_t **a : {&s.tp, &s.tt, &s.gslot, &s.newlab}) {
    HIP_OR_FAIL(&c, dalloc(a, n));
    HIP_OR_FAIL(&c, hipMemsetAsync(*a, 0xff, sizeof(int32_t) * n, c.stream));
  }
  for (int32_t **a : {&s.gcnt, &s.flag}) {
    HIP_OR_FAIL(&c, dalloc(a, n));
    HIP_OR_FAIL(&c, hipMemsetAsync(*a, 0, sizeof(int32_t) * n, c.stream));
  }
  HIP_OR_FAIL(&c, dalloc(&s.jw, n));
  HIP_OR_FAIL(&c, hipMemsetAsync(s.jw, 0, sizeof(unsigned long long) * n, c.stream));
  HIP_OR_FAIL(&c, dalloc(&s.ctr, 4));
  s.ngroups = s.ctr;
  HIP_OR_FAIL(&c, jet::launch_co_prepare(c));
  s.hdeg.resize(n);
  HIP_OR_FAIL(&c, hipMemcpyAsync(s.hdeg.data(), s.deg, sizeof(int64_t) * n, hipMemcpyDeviceToHost, c.stream));
  HIP_OR_FAIL(&c, hipStreamSynchronize(c.stream));
  s.ready = true;
  return JET_OK;
}

// A state whose set-up failed is freed, so a later call starts over.
int co_ensure(Ctx &c) {
  if (c.co && c.co->ready) return JET_OK;
  co_free(c);
  c.co = new jet::CoState();
  const int rc = co_alloc(c);
  if (rc != JET_OK) co_free(c);
  return rc;
}

template <typename T>
void release(T *&p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

// Room for sub-rounds of up to cap vertices, table offsets of len + 1 positions and slots tables.
// A capacity is raised only once its arrays exist; freed arrays are cleared at once.
int co_reserve(Ctx &c, int64_t cap, int64_t ptab_len, int64_t slots) {
  jet::CoState &s = *c.co;
  if (cap > s.cap) {
    s.cap = 0;
    release(s.gpos);
    release(s.gtarget);
    release(s.members);
    release(s.goff);
    release(s.gmoved);
    HIP_OR_FAIL(&c, dalloc(&s.gpos, (size_t)cap));
    HIP_OR_FAIL(&c, dalloc(&s.gtarget, (size_t)cap));
    HIP_OR_FAIL(&c, dalloc(&s.members, (size_t)cap));
    HIP_OR_FAIL(&c, dalloc(&s.goff, (size_t)cap + 1));
    HIP_OR_FAIL(&c, dalloc(&s.gmoved, (size_t)cap));
    s.cap = cap;
  }
  if (ptab_len > s.ptab_len) {
    s.ptab_len = 0;
    release(s.ptab);
    HIP_OR_FAIL(&c, dalloc(&s.ptab, (size_t)ptab_len));
    s.ptab_len = ptab_len;
  }
  if (slots > s.tab_slots) {
    s.tab_slots = 0;
    release(s.tab);
    HIP_OR_FAIL(&c, dalloc(&s.tab, (size_t)slots));
    s.tab_slots = slots;
  }
  return JET_OK;
}

// Sub-rounds `rounds` over the device list d_list (host copy hlist): table offsets, launches.
int co_run(Ctx &c, const int32_t *d_list, const std::vector<int32_t> &hlist,
           const std::vector<std::pair<int64_t, int64_t>> &rounds, int32_t *label, int64_t *cw, int64_t wmax,
           int32_t *t_out) {
  jet::CoState &s = *c.co;
  const int64_t len = (int64_t)hlist.size();
  std::vector<int64_t> P((size_t)len + 1, 0);
  int64_t biggest = 0, longest = 1;
  for (int64_t i = 0; i < len; ++i) {
    const int64_t t = co_table(s.hdeg[(size_t)hlist[(size_t)i]], c.n);
    P[(size_t)i + 1] = P[(size_t)i] + t;
    biggest = std::max(biggest, t);
  }
  for (const auto &r : rounds) longest = std::max(longest, r.second);
  const int64_t slots = std::max<int64_t>(1, std::max(biggest, std::min(P[(size_t)len], c.co_slots)));
  int rc = co_reserve(c, longest, len + 1, slots);
  if (rc != JET_OK) return rc;
  HIP_OR_FAIL(&c, hipMemcpyAsync(s.ptab, P.data(), sizeof(int64_t) * ((size_t)len + 1), hipMemcpyHostToDevice,
                                 c.stream));
  for (const auto &r : rounds) {
    const int64_t end = r.first + r.second;
    for (int64_t a = r.first; a < end;) {
      // the longest run of the sub-round whose tables fit the slots (at least one vertex)
      const int64_t lim = P[(size_t)a] + slots;
      int64_t b = (int64_t)(std::upper_bound(P.begin() + a + 1, P.begin() + end + 1, lim) - P.begin()) - 1;
      b = std::max(b, a + 1);
      HIP_OR_FAIL(&c, jet::launch_co_rate(c, d_list, a, b, P[(size_t)a], label, cw, wmax));
      a = b;
    }
    HIP_OR_FAIL(&c, jet::launch_co_settle(c, d_list + r.first, r.second, label, cw, wmax, t_out));
  }
  return JET_OK;
}

// list[len] (device) holds distinct vertex IDs; its host copy in *host
int co_check_list(Ctx &c, const int32_t *list, int64_t len, const char *what, std::vector<int32_t> *host) {
  jet::CoState &s = *c.co;
  HIP_OR_FAIL(&c, jet::launch_co_check(c, list, len, s.ctr + 1));
  int32_t bad = 0;
  host->resize((size_t)len);
  HIP_OR_FAIL(&c, hipMemcpyAsync(&bad, s.ctr + 1, sizeof(int32_t), hipMemcpyDeviceToHost, c.stream));
  if (len > 0)
    HIP_OR_FAIL(&c, hipMemcpyAsync(host->data(), list, sizeof(int32_t) * (size_t)len, hipMemcpyDeviceToHost,
                                   c.stream));
  HIP_OR_FAIL(&c, hipStreamSynchronize(c.stream));
  if (bad) return fail(&c, JET_EINVAL, std::string(what) + ": " + std::to_string(bad) +
                                           " entries outside [0, n) or repeated");
  return JET_OK;
}

}  // namespace

extern "C" {

void jet_params_default(jet_params *p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->limit = 8;
  p->max_iters = 1000;
  p->num_tau = 3;
  p->tau[0] = 0.75f;
  p->tau[1] = 0.375f;
  p->tau[2] = 0.0f;
  p->deadzone_ppm = 100000;
  p->max_rebalance_rounds = 64;
  p->rb_unweighted = 0;
}

int jet_init(jet_ctx **out, int32_t n, int32_t m, int64_t num_pins, const int64_t *net_offsets, const int32_t *pins,
             const int32_t *net_weights, const int32_t *vertex_weights, int32_t k, double eps, void *stream) {
  g_init_error.clear();
  if (!out) return fail(nullptr, JET_EINVAL, "out is NULL");
  *out = nullptr;
  if (n < 1 || m < 1) return fail(nullptr, JET_EINVAL, "n and m must be >= 1");
  if (num_pins < 1) return fail(nullptr, JET_EINVAL, "num_pins must be >= 1");
  if (num_pins > INT32_MAX) return fail(nullptr, JET_EOVERFLOW, "more than 2^31-1 pins");
  if (k < 2 || k > jet::kMaxK) return fail(nullptr, JET_EINVAL, "k outside [2,128]");
  if (!(eps > 0.0 && eps < 1.0)) return fail(nullptr, JET_EINVAL, "eps outside (0,1)");
  if (!net_offsets || !pins) return fail(nullptr, JET_EINVAL, "net_offsets or pins is NULL");
  jet_ctx *ctx = new (std::nothrow) jet_ctx;
  if (!ctx) return fail(nullptr, JET_ENOMEM, "host allocation failed");
  ctx->c.stream = (hipStream_t)stream;
  ctx->c.k = k;
  ctx->c.eps = eps;
  int rc = init_impl(ctx->c, n, m, num_pins, net_offsets, pins, net_weights, vertex_weights);
  if (rc != JET_OK) {
    g_init_error = ctx->c.last_error;
    if (rc == JET_EHIP && g_init_error.find("out of memory") != std::string::npos) rc = JET_ENOMEM;
    free_ctx(ctx->c);
    delete ctx;
    return rc;
  }
  *out = ctx;
  return JET_OK;
}

int jet_refine_ex(jet_ctx *ctx, int32_t *part, const jet_params *params, jet_stats *stats, jet_trace *trace,
                  int32_t trace_cap, int32_t *trace_len) {
  if (!ctx) return JET_EINVAL;
  ctx->c.last_error.clear();
  return refine_impl(ctx->c, part, params, stats, trace, trace_cap, trace_len);
}

int jet_refine(jet_ctx *ctx, int32_t *part, const jet_params *params, jet_stats *stats) {
  return jet_refine_ex(ctx, part, params, stats, nullptr, 0, nullptr);
}

int jet_rebalance(jet_ctx *ctx, int32_t *part, const jet_params *params, jet_stats *stats) {
  if (!ctx) return JET_EINVAL;
  Ctx &c = ctx->c;
  c.last_error.clear();
  int rc = check_params(c, params, false);
  if (rc != JET_OK) return rc;
  return run_loop(c, part, params, true, stats, nullptr, 0, nullptr);
}

int jet_level_stats(jet_ctx *ctx, const int32_t *part, int64_t out[16]) {
  if (!ctx || !out) return JET_EINVAL;
  Ctx &c = ctx->c;
  c.last_error.clear();
  int rc = build_state(c, part);
  if (rc != JET_OK) return rc;
  HIP_OR_FAIL(&c, jet::launch_level_stats(c, c.lstat));
  int64_t h[5];
  HIP_OR_FAIL(&c, hipMemcpyAsync(h, c.lstat, sizeof h, hipMemcpyDeviceToHost, c.stream));
  HIP_OR_FAIL(&c, hipStreamSynchronize(c.stream));
  const int64_t vals[16] = {c.n, c.m, c.p,  h[3],        c.k,  c.W,  c.lmax, max_block_weight(c),
                            h[0], c.hst->km1, h[2], h[4], h[1], c.A, 0, 0};
  std::memcpy(out, vals, sizeof vals);
  return JET_OK;
}

int jet_tau_features(const int64_t s[16], double eps, int32_t level, int32_t levels, int64_t n_finest,
                     int32_t round, int32_t rounds, double prev_gain, float out[16]) {
  if (!s || !out || levels < 1 || level < 0 || level >= levels || rounds < 1 || round < 0 || round >= rounds ||
      s[0] < 1 || s[1] < 1 || s[2] < 1 || s[3] < 1 || s[4] < 2 || s[6] < 1 || s[10] < 1 || n_finest < s[0])
    return JET_EINVAL;
  const double n = (double)s[0], m = (double)s[1], p = (double)s[2];
  const double f[16] = {std::log2(n),
                        std::log2(m),
                        std::log2(p),
                        p / m,
                        std::log2((double)s[3]),
                        p / n,
                        std::log2((double)s[4]),
                        eps,
                        levels > 1 ? (double)level / (levels - 1) : 0.0,
                        std::log2((double)n_finest / n),
                        (double)s[7] / (double)s[6] - 1.0,
                        (double)s[8] / m,
                        (double)s[9] / (double)s[10],
                        (double)s[11] / n,
                        rounds > 1 ? (double)round / (rounds - 1) : 0.0,
                        prev_gain};
  for (int i = 0; i < 16; ++i) out[i] = (float)f[i];
  return JET_OK;
}

int jet_refine_learned(jet_ctx *ctx, int32_t *part, const jet_params *params, jet_mlp *net, int32_t level,
                       int32_t levels, int64_t n_finest, jet_stats *stats, float *tau_used, int32_t *from_net) {
  if (!ctx) return JET_EINVAL;
  Ctx &c = ctx->c;
  c.last_error.clear();
  int rc = check_params(c, params, true);
  if (rc != JET_OK) return rc;
  float mean[16], sd[16];
  if (net && jet_mlp_get(net, nullptr, mean, sd) != JET_OK)
    return fail(&c, JET_EHIP, std::string("temperature network: ") + jet_mlp_last_error(net));
  jet_stats S;
  std::memset(&S, 0, sizeof S);
  double prev_gain = 0.0;
  for (int r = 0; r < params->num_tau; ++r) {
    float tau = params->tau[r];
    if (from_net) from_net[r] = 0;
    if (net) {
      int64_t st[16];
      float feat[16];
      rc = jet_level_stats(ctx, part, st);
      if (rc != JET_OK) return rc;
      if (jet_tau_features(st, c.eps, level, levels, n_finest, r, params->num_tau, prev_gain, feat) != JET_OK)
        return fail(&c, JET_EINVAL, "level, levels, n_finest or the statistics are out of range");
      bool in_range = true;
      for (int i = 0; i < 16; ++i) in_range = in_range && std::fabs((feat[i] - mean[i]) / sd[i]) <= 6.0f;
      if (in_range) {
        HIP_OR_FAIL(&c, hipMemcpyAsync(c.tau_io, feat, sizeof feat, hipMemcpyHostToDevice, c.stream));
        HIP_OR_FAIL(&c, hipStreamSynchronize(c.stream));  // the network may run on another stream
        float t = 0.0f;
        if (jet::mlp_infer_one(net, c.tau_io, c.tau_io + 16, &t) != JET_OK)
          return fail(&c, JET_EHIP, std::string("temperature network: ") + jet_mlp_last_error(net));
        tau = t;
        if (from_net) from_net[r] = 1;
      }
    }
    if (tau_used) tau_used[r] = tau;
    jet_params one = *params;
    one.num_tau = 1;
    one.tau[0] = tau;
    jet_stats R;
    rc = refine_impl(c, part, &one, &R, nullptr, 0, nullptr);
    if (rc != JET_OK && rc != JET_IMBALANCED) return rc;
    if (r == 0) S.km1_in = R.km1_in;
    S.km1_out = R.km1_out;
    S.lmax = R.lmax;
    S.max_block_weight = R.max_block_weight;
    S.balanced = R.balanced;
    S.iterations += R.iterations;
    S.rebalance_rounds += R.rebalance_rounds;
    S.moves_executed += R.moves_executed;
    S.tau_q_used[r] = R.tau_q_used[0];
    prev_gain = R.km1_in > 0 ? (double)(R.km1_in - R.km1_out) / (double)R.km1_in : 0.0;
  }
  if (stats) *stats = S;
  return S.balanced ? JET_OK : JET_IMBALANCED;
}

int jet_km1(jet_ctx *ctx, const int32_t *part, int64_t *km1) {
  if (!ctx || !km1) return JET_EINVAL;
  ctx->c.last_error.clear();
  int rc = build_state(ctx->c, part);
  if (rc != JET_OK) return rc;
  *km1 = ctx->c.hst->km1;
  return JET_OK;
}

int jet_phi(jet_ctx *ctx, const int32_t *part, int32_t *phi) {
  if (!ctx || !phi) return JET_EINVAL;
  Ctx &c = ctx->c;
  c.last_error.clear();
  if (!part) return fail(&c, JET_EINVAL, "part is NULL");
  HIP_OR_FAIL(&c, jet::launch_check_part(c, part));
  int rc = read_status(c);
  if (rc != JET_OK) return rc;
  HIP_OR_FAIL(&c, jet::launch_build_phi(c, part, phi));
  HIP_OR_FAIL(&c, hipStreamSynchronize(c.stream));
  return JET_OK;
}

int jet_candidates(jet_ctx *ctx, const int32_t *part, const uint8_t *lock, int32_t tau_q, int32_t *t, int32_t *g,
                   uint8_t *in_m) {
  if (!ctx || !t || !g || !in_m) return JET_EINVAL;
  Ctx &c = ctx->c;
  c.last_error.clear();
  if (tau_q < 0 || tau_q > 65536) return fail(&c, JET_EINVAL, "tau_q outside [0,65536]");
  int rc = build_state(c, part);
  if (rc != JET_OK) return rc;
  HIP_OR_FAIL(&c, jet::launch_candidates(c, part, INT32_MIN, lock, tau_q));
  HIP_OR_FAIL(&c, jet::launch_export_candidates(c, t, g, in_m));
  return read_status(c);
}

int jet_afterburner(jet_ctx *ctx, const int32_t *part, const int32_t *t, const int32_t *g, const uint8_t *in_m,
                    int32_t *rg) {
  if (!ctx || !t || !g || !in_m || !rg) return JET_EINVAL;
  Ctx &c = ctx->c;
  c.last_error.clear();
  int rc = build_state(c, part);
  if (rc != JET_OK) return rc;
  HIP_OR_FAIL(&c, jet::launch_reset_counters(c, jet::kResetCandidates | jet::kResetMoves));
  HIP_OR_FAIL(&c, jet::launch_import_candidates(c, part, t, g, in_m));
  rc = read_status(c);
  if (rc != JET_OK) return rc;
  HIP_OR_FAIL(&c, jet::launch_afterburner(c, part));
  HIP_OR_FAIL(&c, hipMemcpyAsync(rg, c.rg, sizeof(int32_t) * (size_t)c.n, hipMemcpyDeviceToDevice, c.stream));
  HIP_OR_FAIL(&c, hipMemsetAsync(c.rg, 0, sizeof(int32_t) * (size_t)c.n, c.stream));
  HIP_OR_FAIL(&c, hipMemsetAsync(c.inm, 0, sizeof(uint32_t) * (((size_t)c.n + 255) / 256 * 8), c.stream));
  return read_status(c);
}

int jet_loop_counts(jet_ctx *ctx, int64_t *host_polls, int64_t *pieces) {
  if (!ctx) return JET_EINVAL;
  if (host_polls) *host_polls = ctx->c.polls;
  if (pieces) *pieces = ctx->c.replays_done;
  return JET_OK;
}

int jet_coarsen(jet_ctx *ctx, const int32_t *order, int64_t max_cluster_weight, int32_t initial_single,
                int32_t cap_div, int32_t *label, int32_t *num_clusters) {
  if (!ctx) return JET_EINVAL;
  Ctx &c = ctx->c;
  c.last_error.clear();
  if (!order || !label) return fail(&c, JET_EINVAL, "order or label is NULL");
  if (c.H > 1) return fail(&c, JET_EUNSUPPORTED, "clustering runs on a single-hypergraph context");
  if (max_cluster_weight < 1) return fail(&c, JET_EINVAL, "max_cluster_weight must be at least 1");
  if (initial_single < 0 || cap_div < 1) return fail(&c, JET_EINVAL, "initial_single < 0 or cap_div < 1");
  int rc = co_ensure(c);
  if (rc != JET_OK) return rc;
  std::vector<int32_t> horder;
  if ((rc = co_check_list(c, order, c.n, "order", &horder)) != JET_OK) return rc;
  jet::CoState &s = *c.co;
  HIP_OR_FAIL(&c, jet::launch_co_init(c, label, s.cw));
  rc = co_run(c, order, horder, co_schedule(c.n, initial_single, cap_div), label, s.cw, max_cluster_weight, nullptr);
  if (rc != JET_OK) return rc;
  HIP_OR_FAIL(&c, jet::launch_co_count(c, label, s.ctr + 2));
  int32_t cnt = 0;
  HIP_OR_FAIL(&c, hipMemcpyAsync(&cnt, s.ctr + 2, sizeof(int32_t), hipMemcpyDeviceToHost, c.stream));
  HIP_OR_FAIL(&c, hipStreamSynchronize(c.stream));
  if (num_clusters) *num_clusters = cnt;
  return JET_OK;
}

int jet_coarsen_subround(jet_ctx *ctx, int32_t *label, int64_t *cw, const int32_t *verts, int32_t count,
                         int64_t max_cluster_weight, int32_t *targets) {
  if (!ctx) return JET_EINVAL;
  Ctx &c = ctx->c;
  c.last_error.clear();
  if (!label || !cw || !targets || (count > 0 && !verts)) return fail(&c, JET_EINVAL, "NULL argument");
  if (c.H > 1) return fail(&c, JET_EUNSUPPORTED, "clustering runs on a single-hypergraph context");
  if (count < 0 || count > c.n) return fail(&c, JET_EINVAL, "count outside [0, n]");
  if (max_cluster_weight < 1) return fail(&c, JET_EINVAL, "max_cluster_weight must be at least 1");
  int rc = co_ensure(c);
  if (rc != JET_OK) return rc;
  if (count == 0) {
    HIP_OR_FAIL(&c, hipMemsetAsync(targets, 0xff, sizeof(int32_t) * (size_t)c.n, c.stream));
    HIP_OR_FAIL(&c, hipStreamSynchronize(c.stream));
    return JET_OK;
  }
  std::vector<int32_t> hverts;
  if ((rc = co_check_list(c, verts, count, "verts", &hverts)) != JET_OK) return rc;
  rc = co_run(c, verts, hverts, {{0, (int64_t)count}}, label, cw, max_cluster_weight, targets);
  if (rc != JET_OK) return rc;
  HIP_OR_FAIL(&c, hipStreamSynchronize(c.stream));
  return JET_OK;
}

namespace {

// common checks of the flow entry points
int flow_args(Ctx &c, const int32_t *part, int32_t a, int32_t b, int32_t alpha) {
  if (!part) return fail(&c, JET_EINVAL, "part is NULL");
  if (c.H > 1) return fail(&c, JET_EUNSUPPORTED, "flow refinement runs on a single-hypergraph context");
  if (a < 0 || b < 0 || a >= c.k || b >= c.k || a == b) return fail(&c, JET_EINVAL, "blocks outside [0,k) or equal");
  if (alpha < 0) return fail(&c, JET_EINVAL, "alpha < 0");
  HIP_OR_FAIL(&c, jet::launch_check_part(c, part));
  return read_status(c);
}

}  // namespace

int jet_flow_region(jet_ctx *ctx, const int32_t *part, int32_t a, int32_t b, int32_t alpha, int8_t *region) {
  if (!ctx) return JET_EINVAL;
  Ctx &c = ctx->c;
  c.last_error.clear();
  if (!region) return fail(&c, JET_EINVAL, "region is NULL");
  int rc = flow_args(c, part, a, b, alpha);
  if (rc != JET_OK) return rc;
  return jet::flow_region(c, part, a, b, alpha, region);
}

int jet_flow_mincut(jet_ctx *ctx, const int32_t *part, int32_t a, int32_t b, const int8_t *term, int64_t *flow,
                    uint8_t *in_sr, uint8_t *in_tr) {
  if (!ctx) return JET_EINVAL;
  Ctx &c = ctx->c;
  c.last_error.clear();
  if (!term || !flow || !in_sr || !in_tr) return fail(&c, JET_EINVAL, "NULL argument");
  int rc = flow_args(c, part, a, b, 0);
  if (rc != JET_OK) return rc;
  return jet::flow_mincut(c, part, a, b, term, flow, in_sr, in_tr);
}

int jet_flow_pair(jet_ctx *ctx, int32_t *part, int32_t a, int32_t b, int32_t alpha, jet_flow_pair_stats *st) {
  if (!ctx) return JET_EINVAL;
  Ctx &c = ctx->c;
  c.last_error.clear();
  int rc = flow_args(c, part, a, b, alpha);
  if (rc != JET_OK) return rc;
  jet::FlowPairResult r;
  rc = jet::flow_pair(c, part, a, b, alpha, &r);
  if (rc != JET_OK) return rc;
  if (st) {
    st->old_cut = r.old_cut;
    st->new_cut = r.new_cut;
    st->iterations = r.iterations;
    st->region_a = r.region_a;
    st->region_b = r.region_b;
    st->moved = r.moved;
    st->replaced = r.replaced;
    st->arcs = r.arcs;
  }
  return JET_OK;
}

int jet_flow_refine(jet_ctx *ctx, int32_t *part, int32_t alpha, int32_t max_rounds, jet_flow_stats *st) {
  if (!ctx) return JET_EINVAL;
  Ctx &c = ctx->c;
  c.last_error.clear();
  if (max_rounds < 0) return fail(&c, JET_EINVAL, "max_rounds < 0");
  int rc = flow_args(c, part, 0, 1, alpha);
  if (rc != JET_OK) return rc;
  jet::FlowRefineResult r;
  rc = jet::flow_refine(c, part, alpha, max_rounds, &r);
  if (rc != JET_OK) return rc;
  if (st) {
    st->km1_in = r.km1_in;
    st->km1_out = r.km1_out;
    st->rounds = r.rounds;
    st->matchings = r.matchings;
    st->pairs = r.pairs;
    st->accepted = r.accepted;
    st->flow_calls = r.flow_calls;
    st->moved = r.moved;
    st->arcs = r.arcs;
  }
  return JET_OK;
}

int jet_rebalance_round(jet_ctx *ctx, int32_t *part, int32_t deadzone_ppm, int32_t *sel_target, int32_t *moved) {
  if (!ctx || !sel_target) return JET_EINVAL;
  Ctx &c = ctx->c;
  c.last_error.clear();
  if (deadzone_ppm < 0 || deadzone_ppm > 1000000) return fail(&c, JET_EINVAL, "deadzone_ppm outside [0,1e6]");
  int64_t A, lmax, dz;
  limits(c.W, c.k, c.eps, deadzone_ppm, &A, &lmax, &dz);
  int rc = build_state(c, part);
  if (rc != JET_OK) return rc;
  HIP_OR_FAIL(&c, hipMemsetAsync(sel_target, 0xff, sizeof(int32_t) * (size_t)c.n, c.stream));
  int32_t mv = 0;
  if (overload(c) > 0) {
    HIP_OR_FAIL(&c, jet::launch_rebalance_round(c, part, dz, sel_target));
    rc = apply_and_read(c, part, 1);
    if (rc != JET_OK) return rc;
    mv = c.hst->n_moves;
  } else {
    HIP_OR_FAIL(&c, hipStreamSynchronize(c.stream));
  }
  if (moved) *moved = mv;
  return JET_OK;
}

int jet_prof_enable(jet_ctx *ctx, int32_t on) {
  if (!ctx) return JET_EINVAL;
  Ctx &c = ctx->c;
  HIP_OR_FAIL(&c, hipMemsetAsync(c.dprof, 0, sizeof(jet::DevProf), c.stream));
  HIP_OR_FAIL(&c, hipStreamSynchronize(c.stream));
  if (c.prof != (on != 0)) drop_graph(c);  // the marks are part of the captured iteration
  c.prof = on != 0;
  return JET_OK;
}

int jet_prof_read(jet_ctx *ctx, jet_prof_entry *out, int32_t cap, int32_t *count) {
  if (!ctx || (!out && cap > 0)) return JET_EINVAL;
  Ctx &c = ctx->c;
  jet::DevProf dp;
  HIP_OR_FAIL(&c, hipMemcpyAsync(&dp, c.dprof, sizeof dp, hipMemcpyDeviceToHost, c.stream));
  HIP_OR_FAIL(&c, hipStreamSynchronize(c.stream));
  static const char *names[jet::kProfFamilies] = {"candidates",   "candidates_hub", "afterburner", "select_moves",
                                                  "apply",        "rebalance_gain", "rebalance_select"};
  int32_t cnt = 0;
  for (int f = 0; f < jet::kProfFamilies; ++f) {
    if (dp.launches[f] == 0) continue;
    if (cnt < cap) {
      std::memset(out[cnt].name, 0, sizeof out[cnt].name);
      std::strncpy(out[cnt].name, names[f], sizeof out[cnt].name - 1);
      out[cnt].launches = (int64_t)dp.launches[f];
      out[cnt].total_ms = (double)dp.ticks[f] / c.wall_khz;
      out[cnt].alg_bytes = dp.bytes[f];
    }
    ++cnt;
  }
  if (count) *count = cnt;
  return JET_OK;
}

int jet_set_option(jet_ctx *ctx, int32_t option, int64_t value) {
  if (!ctx) return JET_EINVAL;
  Ctx &c = ctx->c;
  drop_graph(c);  // launch arguments of the captured iteration may change
  switch (option) {
  case JET_OPT_APPLY_DIVISOR:
    if (value < 0 || value > (1 << 20)) return fail(&c, JET_EINVAL, "apply divisor outside [0, 2^20]");
    c.apply_divisor = (int32_t)value;
    return JET_OK;
  case JET_OPT_APPLY_WIDE:
    if (value < 0 || value > 1) return fail(&c, JET_EINVAL, "apply wide option must be 0 or 1");
    c.wide_enabled = value != 0;
    return JET_OK;
  case JET_OPT_CAND_LANE_DEGREE:
    if (value < 0 || value > (1 << 20)) return fail(&c, JET_EINVAL, "lane degree outside [0, 2^20]");
    c.lane_degree = (int32_t)value;
    return JET_OK;
  case JET_OPT_SEL_SPLIT_MIN:
    if (value < 0 || value > ((int64_t)1 << 31) - 1) return fail(&c, JET_EINVAL, "split threshold outside [0, 2^31)");
    c.sel_split_min = (int32_t)value;
    return JET_OK;
  case JET_OPT_PROF_FAMILIES:
    if (value < 0 || value >= (int64_t)1 << jet::kProfFamilies)
      return fail(&c, JET_EINVAL, "profiled family mask outside [0, 2^7)");
    c.prof_mask = (uint32_t)value;
    return JET_OK;
  case JET_OPT_GRAPH:
    if (value < 0 || value > 1) return fail(&c, JET_EINVAL, "graph option must be 0 or 1");
    c.use_graph = value != 0;
    return JET_OK;
  case JET_OPT_RB_SLOTS:
    if (value < 1 || value > 64) return fail(&c, JET_EINVAL, "rebalancing slots outside [1, 64]");
    c.rb_slots = (int32_t)value;
    return JET_OK;
  case JET_OPT_REPLAYS:
    if (value < 1 || value > 1024) return fail(&c, JET_EINVAL, "replays per poll outside [1, 1024]");
    c.replays = (int32_t)value;
    return JET_OK;
  case JET_OPT_GRID:
    if (value < 64 || value > 65536) return fail(&c, JET_EINVAL, "persistent grid outside [64, 65536]");
    c.grid_cap = value;
    return JET_OK;
  case JET_OPT_CAND_XCD:
    if (value < 0 || value > 1) return fail(&c, JET_EINVAL, "XCD option must be 0 or 1");
    c.cand_xcd = (int32_t)value;
    return JET_OK;
  case JET_OPT_APPLY_XCD:
    if (value < 0 || value > 1) return fail(&c, JET_EINVAL, "XCD option must be 0 or 1");
    c.apply_xcd = (int32_t)value;
    return JET_OK;
  case JET_OPT_FLOW_WORKERS:
    if (value < 1 || value > 8) return fail(&c, JET_EINVAL, "flow workers outside [1, 8]");
    c.flow_workers = (int32_t)value;
    return JET_OK;
  case JET_OPT_GRAPH_KERNELS:
    if (value < 0 || value > 1) return fail(&c, JET_EINVAL, "graph kernel option must be 0 or 1");
    c.graph_kernels = (int32_t)value;
    return JET_OK;
  case JET_OPT_RB_XCD:
    if (value < 0 || value > 1) return fail(&c, JET_EINVAL, "XCD option must be 0 or 1");
    c.rb_xcd = (int32_t)value;
    return JET_OK;
  case JET_OPT_CO_TABLE_SLOTS:
    if (value < 16 || value > ((int64_t)1 << 31)) return fail(&c, JET_EINVAL, "table slots outside [16, 2^31]");
    c.co_slots = value;
    return JET_OK;
  default: return fail(&c, JET_EINVAL, "unknown option " + std::to_string(option));
  }
}

int jet_free(jet_ctx *ctx) {
  if (!ctx) return JET_OK;
  (void)hipStreamSynchronize(ctx->c.stream);
  free_ctx(ctx->c);
  delete ctx;
  return JET_OK;
}

const char *jet_strerror(int code) {
  switch (code) {
  case JET_OK: return "ok";
  case JET_IMBALANCED: return "completed, but the partition violates the balance constraint";
  case JET_EINVAL: return "invalid argument";
  case JET_ENOMEM: return "out of memory";
  case JET_EHIP: return "HIP runtime error";
  case JET_EOVERFLOW: return "integer range exceeded";
  case JET_EUNSUPPORTED: return "input shape not supported by this library";
  default: return "unknown error";
  }
}

const char *jet_last_error(const jet_ctx *ctx) {
  return ctx ? ctx->c.last_error.c_str() : g_init_error.c_str();
}


// ---- batches: one context per hypergraph; lanes of streams, each driven by a host thread, take
// the hypergraphs largest first.  A hypergraph's result depends only on its own inputs.

struct jet_batch {
  std::vector<jet_ctx *> uctx;          // union contexts: hypergraphs of one k, concatenated
  std::vector<int32_t> ctx_of, hg_of;   // per hypergraph: its union context and its index there
  std::vector<std::vector<int32_t>> members;  // per union context: the hypergraphs, in its order
  hipStream_t caller = nullptr;
  hipStream_t gstream = nullptr;        // capture stream of the batch graph
  hipGraph_t graph = nullptr;           // one full iteration of every union context
  hipGraphExec_t gexec = nullptr;
  bool use_graph = true;
  int64_t polls = 0, replays_done = 0;
  std::string last_error;
};

static int batch_fail(jet_batch *b, int code, const std::string &msg) {
  if (b) b->last_error = msg;
  else g_init_error = msg;
  return code;
}

static void batch_drop_graph(jet_batch *b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
}

namespace {

struct HostHg {
  int32_t n = 0, m = 0, k = 0;
  int64_t p = 0, W = 0;
  double eps = 0.0;
  std::vector<int64_t> off;
  std::vector<int32_t> pins, nw, vw;
};

// Copies one hypergraph to the host and checks what a union cannot check for it (pins inside its
// own vertex range, offsets, weights, its total weight).
int load_hg(const jet_hg_desc &d, HostHg &h, std::string &msg) {
  if (d.n < 1 || d.m < 1 || d.num_pins < 1) return msg = "n, m and num_pins must be >= 1", JET_EINVAL;
  if (d.num_pins > INT32_MAX) return msg = "more than 2^31-1 pins", JET_EOVERFLOW;
  if (d.k < 2 || d.k > jet::kMaxK) return msg = "k outside [2,128]", JET_EINVAL;
  if (!(d.eps > 0.0 && d.eps < 1.0)) return msg = "eps outside (0,1)", JET_EINVAL;
  if (!d.net_offsets || !d.pins) return msg = "net_offsets or pins is NULL", JET_EINVAL;
  h.n = d.n;
  h.m = d.m;
  h.p = d.num_pins;
  h.k = d.k;
  h.eps = d.eps;
  h.off.resize((size_t)d.m + 1);
  h.pins.resize((size_t)d.num_pins);
  hipError_t e = hipMemcpy(h.off.data(), d.net_offsets, sizeof(int64_t) * h.off.size(), hipMemcpyDefault);
  if (e == hipSuccess) e = hipMemcpy(h.pins.data(), d.pins, sizeof(int32_t) * h.pins.size(), hipMemcpyDefault);
  if (e == hipSuccess && d.net_weights) {
    h.nw.resize((size_t)d.m);
    e = hipMemcpy(h.nw.data(), d.net_weights, sizeof(int32_t) * h.nw.size(), hipMemcpyDefault);
  }
  if (e == hipSuccess && d.vertex_weights) {
    h.vw.resize((size_t)d.n);
    e = hipMemcpy(h.vw.data(), d.vertex_weights, sizeof(int32_t) * h.vw.size(), hipMemcpyDefault);
  }
  if (e != hipSuccess) return msg = std::string("copy: ") + hipGetErrorString(e), JET_EHIP;
  if (h.off[0] != 0 || h.off[(size_t)d.m] != d.num_pins)
    return msg = "net_offsets must start at 0 and end at num_pins", JET_EINVAL;
  for (int32_t x = 0; x < d.m; ++x)
    if (h.off[x + 1] <= h.off[x]) return msg = "net " + std::to_string(x) + " is empty or offsets decrease", JET_EINVAL;
  for (int64_t q = 0; q < d.num_pins; ++q)
    if (h.pins[q] < 0 || h.pins[q] >= d.n) return msg = "pin at index " + std::to_string(q) + " outside [0,n)", JET_EINVAL;
  for (int32_t w : h.nw)
    if (w < 1) return msg = "a vertex or net weight is below 1", JET_EINVAL;
  int64_t W = 0;
  for (int32_t w : h.vw) {
    if (w < 1) return msg = "a vertex or net weight is below 1", JET_EINVAL;
    W += w;
  }
  h.W = h.vw.empty() ? (int64_t)d.n : W;
  if (h.W > INT32_MAX) return msg = "total vertex weight reaches 2^31", JET_EOVERFLOW;
  return JET_OK;
}

// One union context over hypergraphs `ids` (same k): concatenated CSR, vertex and net owners,
// per-hypergraph limits and loop records.
int make_union(const std::vector<HostHg> &hh, const std::vector<int32_t> &ids, hipStream_t stream, jet_ctx **out,
               std::string &msg) {
  const int32_t k = hh[ids[0]].k;
  int64_t n = 0, m = 0, p = 0;
  bool any_nw = false, any_vw = false;
  for (int32_t i : ids) {
    n += hh[i].n;
    m += hh[i].m;
    p += hh[i].p;
    any_nw = any_nw || !hh[i].nw.empty();
    any_vw = any_vw || !hh[i].vw.empty();
  }
  std::vector<int64_t> off;
  std::vector<int32_t> pins, nw, vw;
  std::vector<uint16_t> vhg, nhg;
  off.reserve((size_t)m + 1);
  pins.reserve((size_t)p);
  off.push_back(0);
  jet_ctx *ctx = new (std::nothrow) jet_ctx;
  if (!ctx) return msg = "host allocation failed", JET_ENOMEM;
  Ctx &c = ctx->c;
  c.stream = stream;
  c.k = k;
  c.eps = hh[ids[0]].eps;
  c.H = (int32_t)ids.size();
  // every hypergraph's vertices start on a tile; the padding vertices up to the next start belong
  // to the pseudo-hypergraph H (no nets, block 0, never in a phase)
  int64_t v0 = 0, e0 = 0;
  any_vw = true;  // padding vertices need a weight of their own: every vertex gets one
  for (size_t h = 0; h < ids.size(); ++h) {
    const HostHg &g = hh[ids[h]];
    c.hg_v0.push_back((int32_t)v0);
    c.hg_n.push_back(g.n);
    c.hg_e0.push_back((int32_t)e0);
    for (int32_t e = 0; e < g.m; ++e) off.push_back(off.back() + (g.off[e + 1] - g.off[e]));
    for (int32_t x : g.pins) pins.push_back((int32_t)(x + v0));
    if (any_nw)
      for (int32_t e = 0; e < g.m; ++e) nw.push_back(g.nw.empty() ? 1 : g.nw[e]);
    for (int32_t v = 0; v < g.n; ++v) vw.push_back(g.vw.empty() ? 1 : g.vw[v]);
    const int64_t padded = (g.n + jet::kUnionTile - 1) / jet::kUnionTile * jet::kUnionTile;
    for (int64_t v = g.n; v < padded; ++v) vw.push_back(1);
    vhg.insert(vhg.end(), (size_t)g.n, (uint16_t)h);
    vhg.insert(vhg.end(), (size_t)(padded - g.n), (uint16_t)ids.size());
    nhg.insert(nhg.end(), (size_t)g.m, (uint16_t)h);
    e0 += g.m;
    n += padded - g.n;
    v0 += padded - g.n;
    int64_t A, lmax, dz;
    limits(g.W, k, g.eps, 0, &A, &lmax, &dz);
    c.hg_W.push_back(g.W);
    c.hg_A.push_back(A);
    c.hg_lmax.push_back(lmax);
    c.hg_eps.push_back(g.eps);
    v0 += g.n;
  }
  c.hg_v0.push_back((int32_t)v0);
  c.hg_e0.push_back((int32_t)e0);
  int rc = init_impl(c, (int32_t)n, (int32_t)m, p, off.data(), pins.data(), any_nw ? nw.data() : nullptr,
                     any_vw ? vw.data() : nullptr);
  if (rc == JET_OK) {
    hipError_t e = dalloc(&c.vhg, vhg.size());
    if (e == hipSuccess) e = dalloc(&c.nhg, nhg.size());
    if (e == hipSuccess) e = hipMemcpy(c.vhg, vhg.data(), sizeof(uint16_t) * vhg.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c.nhg, nhg.data(), sizeof(uint16_t) * nhg.size(), hipMemcpyHostToDevice);
    // padding vertices stay in block 0 of the pseudo-hypergraph
    if (e == hipSuccess) e = hipMemset(c.cpart, 0, sizeof(int32_t) * (size_t)c.n);
    // H + 1 records: the pseudo-hypergraph of the padding vertices is never in a phase
    if (e == hipSuccess) e = dalloc(&c.lcs, (size_t)c.H + 1);
    if (e == hipSuccess) e = hipHostMalloc((void **)&c.hlcs, sizeof(jet::LoopCtl) * ((size_t)c.H + 1));
    if (e == hipSuccess) {
      std::memset(c.hlcs, 0, sizeof(jet::LoopCtl) * ((size_t)c.H + 1));
      c.hlcs[c.H].phase = jet::kPhDone;
      c.hlcs[c.H].phase_mask = 1 << jet::kPhDone;
      e = hipMemcpy(c.lcs, c.hlcs, sizeof(jet::LoopCtl) * ((size_t)c.H + 1), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) rc = fail_hip(&c, e, "union set-up");
  }
  if (rc != JET_OK) {
    msg = c.last_error;
    free_ctx(c);
    delete ctx;
    return rc;
  }
  *out = ctx;
  return JET_OK;
}

// the hypergraph of union vertex v (for error messages)
int32_t hg_of_vertex(const Ctx &c, int64_t v) {
  return (int32_t)(std::upper_bound(c.hg_v0.begin(), c.hg_v0.end(), (int32_t)v) - c.hg_v0.begin()) - 1;
}

}  // namespace

int jet_batch_init(jet_batch **out, int32_t count, const jet_hg_desc *descs, void *stream) {
  g_init_error.clear();
  if (!out) return batch_fail(nullptr, JET_EINVAL, "out is NULL");
  *out = nullptr;
  if (count < 1 || !descs) return batch_fail(nullptr, JET_EINVAL, "count < 1 or descs is NULL");
  std::vector<HostHg> hh((size_t)count);
  for (int32_t i = 0; i < count; ++i) {
    std::string msg;
    const int rc = load_hg(descs[i], hh[i], msg);
    if (rc != JET_OK) return batch_fail(nullptr, rc, "hypergraph " + std::to_string(i) + ": " + msg);
  }
  jet_batch *b = new (std::nothrow) jet_batch;
  if (!b) return batch_fail(nullptr, JET_ENOMEM, "host allocation failed");
  b->caller = (hipStream_t)stream;
  b->ctx_of.assign((size_t)count, -1);
  b->hg_of.assign((size_t)count, -1);
  if (const char *env = std::getenv("JET_GRAPH")) b->use_graph = std::atoi(env) != 0;
  // one union per k (in input order), split where a union would exceed its limits
  for (int32_t k = 2; k <= jet::kMaxK; ++k) {
    std::vector<int32_t> ids;
    int64_t n = 0, m = 0, p = 0;
    auto flush = [&]() -> int {
      if (ids.empty()) return JET_OK;
      jet_ctx *u = nullptr;
      std::string msg;
      const int rc = make_union(hh, ids, (hipStream_t)stream, &u, msg);
      if (rc != JET_OK) {
        std::string which;
        for (int32_t i : ids) which += (which.empty() ? "" : ",") + std::to_string(i);
        return batch_fail(nullptr, rc, "hypergraphs " + which + ": " + msg);
      }
      for (size_t h = 0; h < ids.size(); ++h) {
        b->ctx_of[ids[h]] = (int32_t)b->uctx.size();
        b->hg_of[ids[h]] = (int32_t)h;
      }
      b->uctx.push_back(u);
      b->members.push_back(ids);
      ids.clear();
      n = m = p = 0;
      return JET_OK;
    };
    for (int32_t i = 0; i < count; ++i) {
      if (hh[i].k != k) continue;
      // room for this hypergraph and the padding's pseudo-hypergraph; vertices counted with padding
      const int64_t padded = (hh[i].n + jet::kUnionTile - 1) / jet::kUnionTile * jet::kUnionTile;
      const bool full = !ids.empty() &&
                        ((int64_t)(ids.size() + 2) > jet::kMaxH || (int64_t)(ids.size() + 2) * k > jet::kMaxSeg ||
                         n + padded > INT32_MAX || m + hh[i].m > INT32_MAX || p + hh[i].p > INT32_MAX);
      if (full) {
        const int rc = flush();
        if (rc != JET_OK) {
          jet_batch_free(b);
          return rc;
        }
      }
      ids.push_back(i);
      n += padded;
      m += hh[i].m;
      p += hh[i].p;
    }
    const int rc = flush();
    if (rc != JET_OK) {
      jet_batch_free(b);
      return rc;
    }
  }
  *out = b;
  return JET_OK;
}

int jet_batch_set_option(jet_batch *b, int32_t option, int64_t value) {
  if (!b) return JET_EINVAL;
  batch_drop_graph(b);
  if (option == JET_OPT_GRAPH) {
    if (value < 0 || value > 1) return batch_fail(b, JET_EINVAL, "graph option must be 0 or 1");
    b->use_graph = value != 0;
    return JET_OK;
  }
  for (size_t i = 0; i < b->uctx.size(); ++i) {
    int rc = jet_set_option(b->uctx[i], option, value);
    if (rc != JET_OK) return batch_fail(b, rc, b->uctx[i]->c.last_error);
  }
  return JET_OK;
}

int jet_batch_refine(jet_batch *b, int32_t *const *parts, const jet_params *params, int32_t replays,
                     jet_stats *stats, int32_t *rcs) {
  if (!b || !parts || !params) return JET_EINVAL;
  if (replays < 1 || replays > 1024) return batch_fail(b, JET_EINVAL, "replays outside [1, 1024]");
  b->last_error.clear();
  const int32_t count = (int32_t)b->ctx_of.size();
  for (int32_t i = 0; i < count; ++i)
    if (!parts[i]) return batch_fail(b, JET_EINVAL, "hypergraph " + std::to_string(i) + ": part is NULL");
  hipStream_t s = b->caller;
  // partitions in, state built, loop records written and completed
  for (jet_ctx *u : b->uctx) {
    Ctx &c = u->c;
    c.stream = s;
    c.last_error.clear();
    int rc = check_params(c, params, true);
    if (rc != JET_OK) return batch_fail(b, rc, c.last_error);
  }
  for (int32_t i = 0; i < count; ++i) {
    Ctx &c = b->uctx[b->ctx_of[i]]->c;
    const int32_t h = b->hg_of[i];
    const hipError_t e = hipMemcpyAsync(c.cpart + c.hg_v0[h], parts[i], sizeof(int32_t) * (size_t)c.hg_n[h],
                                        hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return batch_fail(b, JET_EHIP, std::string("partition copy: ") + hipGetErrorString(e));
  }
  for (size_t ui = 0; ui < b->uctx.size(); ++ui) {
    Ctx &c = b->uctx[ui]->c;
    const int32_t bad = -1;
    c.hst->err_arg = bad;
    int rc = build_state(c, c.cpart);
    if (rc != JET_OK) {
      std::string msg = c.last_error;
      if (msg.find("part[") == 0) {  // name the hypergraph and its own vertex
        const int64_t v = std::atoll(msg.c_str() + 5);
        const int32_t h = hg_of_vertex(c, v);
        if (h >= 0 && h < c.H)
          msg = "hypergraph " + std::to_string(b->members[ui][h]) + ": part[" + std::to_string(v - c.hg_v0[h]) +
                "] outside [0,k)";
      }
      return batch_fail(b, rc, msg);
    }
    for (int32_t h = 0; h < c.H; ++h) {
      int64_t A, lmax, dz;
      limits(c.hg_W[h], c.k, c.hg_eps[h], params->deadzone_ppm, &A, &lmax, &dz);
      fill_record(c.hlcs[h], *params, false, 0, lmax, dz, A);
    }
    hipError_t e = hipMemcpyAsync(c.lcs, c.hlcs, sizeof(jet::LoopCtl) * (size_t)c.H, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = jet::launch_loop_init(c);
    if (e == hipSuccess)
      e = hipMemcpyAsync(c.best, c.cpart, sizeof(int32_t) * (size_t)c.n, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return batch_fail(b, JET_EHIP, std::string("loop set-up: ") + hipGetErrorString(e));
  }
  // the whole batch's iteration as one graph: every union context's launches, one after another
  if (b->use_graph && !b->gexec) {
    if (!b->gstream) {
      const hipError_t e = hipStreamCreateWithFlags(&b->gstream, hipStreamNonBlocking);
      if (e != hipSuccess) return batch_fail(b, JET_EHIP, std::string("stream: ") + hipGetErrorString(e));
    }
    hipError_t e = hipStreamBeginCapture(b->gstream, hipStreamCaptureModeThreadLocal);
    hipError_t le = hipSuccess;
    if (e == hipSuccess) {
      for (jet_ctx *u : b->uctx) {
        u->c.stream = b->gstream;
        if (le == hipSuccess) le = jet::launch_tick(u->c, jet::kTickAll);
        u->c.stream = s;
      }
      e = hipStreamEndCapture(b->gstream, &b->graph);
    }
    if (e == hipSuccess && le == hipSuccess) e = hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess || le != hipSuccess) {
      batch_drop_graph(b);
      return batch_fail(b, JET_EHIP, std::string("capturing the batch graph: ") +
                                         hipGetErrorString(e != hipSuccess ? e : le));
    }
  }
  int64_t cap = 16;
  for (jet_ctx *u : b->uctx)
    cap = std::max<int64_t>(cap, (int64_t)params->num_tau * ((int64_t)params->max_iters + 2) *
                                     ((int64_t)params->max_rebalance_rounds / std::max(1, u->c.rb_slots) + 3) + 16);
  int64_t ticks = 0;
  b->polls = 0;
  for (;;) {
    for (int32_t g = 0; g < replays; ++g) {
      hipError_t e = hipSuccess;
      if (b->use_graph) e = hipGraphLaunch(b->gexec, s);
      else
        for (jet_ctx *u : b->uctx)
          if (e == hipSuccess) e = jet::launch_tick(u->c, jet::kTickAll);
      if (e != hipSuccess) return batch_fail(b, JET_EHIP, std::string("launch: ") + hipGetErrorString(e));
    }
    ticks += replays;
    bool done = true;
    for (jet_ctx *u : b->uctx) {
      Ctx &c = u->c;
      const hipError_t e = hipMemcpyAsync(c.hlcs, c.lcs, sizeof(jet::LoopCtl) * (size_t)c.H, hipMemcpyDeviceToHost, s);
      if (e != hipSuccess) return batch_fail(b, JET_EHIP, std::string("poll: ") + hipGetErrorString(e));
      const int rc = read_status(c);
      if (rc != JET_OK) return batch_fail(b, rc, c.last_error);
      for (int32_t h = 0; h < c.H && done; ++h) done = c.hlcs[h].phase == jet::kPhDone;
    }
    b->polls += 1;
    if (done) break;
    if (ticks > cap) return batch_fail(b, JET_EHIP, "the batch loop did not finish within its bound");
  }
  b->replays_done = ticks;
  // partitions out, statistics per hypergraph
  int result = JET_OK;
  for (int32_t i = 0; i < count; ++i) {
    Ctx &c = b->uctx[b->ctx_of[i]]->c;
    const int32_t h = b->hg_of[i];
    const hipError_t e = hipMemcpyAsync(parts[i], c.cpart + c.hg_v0[h], sizeof(int32_t) * (size_t)c.hg_n[h],
                                        hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return batch_fail(b, JET_EHIP, std::string("partition copy: ") + hipGetErrorString(e));
    const jet::LoopCtl &r = c.hlcs[h];
    jet_stats S;
    std::memset(&S, 0, sizeof S);
    S.km1_in = r.km1_in;
    S.km1_out = r.km1;
    S.lmax = r.lmax;
    int64_t mx = 0;
    for (int32_t bb = 0; bb < c.k; ++bb) mx = std::max(mx, c.hst->bw[(int64_t)h * c.k + bb]);
    S.max_block_weight = mx;
    S.balanced = mx <= r.lmax;
    S.iterations = r.iterations;
    S.rebalance_rounds = r.rebalance_rounds;
    S.moves_executed = r.moves_executed;
    for (int t = 0; t < params->num_tau; ++t) S.tau_q_used[t] = quantize_tau(params->tau[t]);
    if (stats) stats[i] = S;
    const int rc = S.balanced ? JET_OK : JET_IMBALANCED;
    if (rcs) rcs[i] = rc;
    if (rc == JET_IMBALANCED) result = JET_IMBALANCED;
  }
  const hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return batch_fail(b, JET_EHIP, std::string("sync: ") + hipGetErrorString(e));
  return result;
}

int jet_batch_free(jet_batch *b) {
  if (!b) return JET_OK;
  (void)hipStreamSynchronize(b->caller);
  batch_drop_graph(b);
  if (b->gstream) (void)hipStreamDestroy(b->gstream);
  for (jet_ctx *u : b->uctx) jet_free(u);
  delete b;
  return JET_OK;
}

int jet_batch_prof_enable(jet_batch *b, int32_t on) {
  if (!b) return JET_EINVAL;
  batch_drop_graph(b);
  for (jet_ctx *u : b->uctx) {
    const int rc = jet_prof_enable(u, on);
    if (rc != JET_OK) return batch_fail(b, rc, u->c.last_error);
  }
  return JET_OK;
}

int jet_batch_prof_read(jet_batch *b, jet_prof_entry *out, int32_t cap, int32_t *count) {
  if (!b || (!out && cap > 0)) return JET_EINVAL;
  std::vector<jet_prof_entry> sum;
  for (jet_ctx *u : b->uctx) {
    jet_prof_entry e[jet::kProfFamilies];
    int32_t n = 0;
    const int rc = jet_prof_read(u, e, jet::kProfFamilies, &n);
    if (rc != JET_OK) return batch_fail(b, rc, u->c.last_error);
    for (int32_t i = 0; i < n; ++i) {
      auto it = std::find_if(sum.begin(), sum.end(),
                             [&](const jet_prof_entry &x) { return std::strcmp(x.name, e[i].name) == 0; });
      if (it == sum.end()) {
        sum.push_back(e[i]);
      } else {
        it->launches += e[i].launches;
        it->total_ms += e[i].total_ms;
        it->alg_bytes += e[i].alg_bytes;
      }
    }
  }
  for (int32_t i = 0; i < (int32_t)sum.size() && i < cap; ++i) out[i] = sum[i];
  if (count) *count = (int32_t)sum.size();
  return JET_OK;
}

const char *jet_batch_last_error(const jet_batch *b) { return b ? b->last_error.c_str() : g_init_error.c_str(); }

}  // extern "C"
