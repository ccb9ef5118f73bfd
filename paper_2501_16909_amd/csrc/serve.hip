// Continuous-batching colocation loop and its admission rule.
//
// The paper asks a colocation scheduler to decide per kernel, to predict
// each kernel's slowdown from its per-resource sensitivity and the
// co-runners' pressure, and to trade a bounded slowdown for utilisation
// (Section 5.1); it shows single-metric rules (summed achieved occupancy,
// Section 3 Pitfall 1) mispredicting.  serve_run admits arriving requests
// FIFO under one of three rules (memory only, summed occupancy, predicted
// slowdown) and runs admitted requests concurrently on slot streams.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"
#include "runtime.h"

using namespace ci;

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

const ci_profile_t* profile_of(const ci_policy_t* p, int kind) {
  for (int i = 0; i < p->nprofiles; ++i)
    if (p->profiles[i].kind == kind) return &p->profiles[i];
  return nullptr;
}

// Piecewise-linear slowdown curve at intensity x (points at 0, .25, .5, .75, 1).
double curve_at(const float* s, double x) {
  x = std::min(1.0, std::max(0.0, x));
  const double pos = x * (CI_NPOINTS - 1);
  int i = (int)std::floor(pos);
  if (i >= CI_NPOINTS - 1) return s[CI_NPOINTS - 1];
  const double t = pos - i;
  return (double)s[i] + ((double)s[i + 1] - (double)s[i]) * t;  // in FP64, not the FP32 difference
}

bool has_read_curve(const ci_profile_t* p) {
  for (int i = 0; i < CI_NPOINTS; ++i)
    if (p->sens_hbm_read[i] != 0.0f) return true;
  return false;
}

// The estimator (see ci_predict_slowdown in coloc.h).
double predict_one(const ci_profile_t* v, const ci_profile_t* const* co, int nco) {
  const bool split = has_read_curve(v);
  double press[CI_RES_COUNT] = {};
  double press_read = 0.0;
  for (int o = 0; o < nco; ++o) {
    for (int r = 0; r < CI_RES_COUNT; ++r) {
      if (r == CI_RES_HBM && split && co[o]->hbm_write_frac < CI_READ_MOSTLY_WRITE_FRAC)
        press_read += co[o]->press_hbm_read;
      else
        press[r] += co[o]->press[r];
    }
  }
  double out = 1.0;
  for (int r = 0; r < CI_RES_COUNT; ++r) out *= std::max(1.0, curve_at(v->sens[r], press[r]));
  if (split) out *= std::max(1.0, curve_at(v->sens_hbm_read, press_read));
  return out;
}

// Predicted slowdown of job `j` beside every other job of `group` and the
// background load `bg` (if any).
double predict(const std::vector<const ci_profile_t*>& group, size_t j, const ci_profile_t* bg) {
  std::vector<const ci_profile_t*> co;
  for (size_t o = 0; o < group.size(); ++o)
    if (o != j) co.push_back(group[o]);
  if (bg) co.push_back(bg);
  return predict_one(group[j], co.data(), (int)co.size());
}

// First-fit allocator over one device arena (offsets in bytes, 256-aligned).
class Arena {
 public:
  explicit Arena(uint64_t size) { free_[0] = size; }
  bool alloc(uint64_t bytes, uint64_t* off) {
    bytes = (bytes + 255) & ~255ull;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const uint64_t rest = it->second - bytes, at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(uint64_t off, uint64_t bytes) {
    bytes = (bytes + 255) & ~255ull;
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  uint64_t largest_free() const {
    uint64_t m = 0;
    for (auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }
  uint64_t used() const { return used_; }

 private:
  uint64_t used_ = 0;
  std::map<uint64_t, uint64_t> free_;
};

uint64_t elem_bytes(int dt) { return dt == CI_DT_F32 ? 4 : dt == CI_DT_BF16 ? 2 : 1; }

// Bytes a request holds while it runs: operands, output and one FP32
// staging buffer its inputs are drawn into before conversion.
uint64_t footprint(const ci_request_t& q) {
  auto al = [](uint64_t b) { return (b + 255) & ~255ull; };
  switch (q.kind) {
    case CI_VICTIM_TRIAD_F32: return 3 * al(q.n * 4);
    case CI_VICTIM_GEMM: {
      const uint64_t e = elem_bytes(q.dtype);
      uint64_t stage = std::max(q.m, q.n) * q.k * 4;
      if (q.dtype == CI_DT_F32) stage = 0;
      return al(q.m * q.k * e) + al(q.n * q.k * e) + al(q.m * q.n * 4) + al(stage);
    }
    case CI_VICTIM_GEMV: return al(q.n * q.k * 2) + al(q.k * 2) + al(q.n * 4) + al(std::max(q.n * q.k, q.k) * 4);
    default: return 0;
  }
}

struct Running {
  int idx = -1;
  uint64_t off = 0, bytes = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, done = nullptr;
  ci_victim_desc_t d{};
};

}  // namespace

extern "C" ci_status_t ci_predict_slowdown(const ci_profile_t* victim,
                                           const ci_profile_t* const* corunners, int nco,
                                           double* out) {
  if (!victim || !out || nco < 0 || (nco && !corunners))
    return set_err(CI_ERR_INVALID_ARG, "ci_predict_slowdown: bad argument");
  for (int o = 0; o < nco; ++o)
    if (!corunners[o]) return set_err(CI_ERR_INVALID_ARG, "ci_predict_slowdown: co-runner %d is NULL", o);
  *out = predict_one(victim, corunners, nco);
  return CI_OK;
}

extern "C" ci_status_t ci_admit(const ci_policy_t* p, const int* running_kinds, int nrun,
                                int cand_kind, uint64_t cand_bytes, uint64_t free_bytes,
                                int* admit) {
  if (!p || !admit || nrun < 0 || (nrun && !running_kinds))
    return set_err(CI_ERR_INVALID_ARG, "ci_admit: bad argument");
  if (p->kind != CI_POLICY_NAIVE && p->kind != CI_POLICY_USHER && p->kind != CI_POLICY_SENSITIVITY)
    return set_err(CI_ERR_INVALID_ARG, "ci_admit: policy %d", p->kind);
  *admit = 0;
  if (cand_bytes > free_bytes || nrun >= p->slots) return CI_OK;
  // Memory and a slot are all a request needs on an idle device: the
  // occupancy and slowdown rules bound colocation (nothing would ever free
  // up for a lone request they refuse, and the loop would wait forever).
  if (p->kind == CI_POLICY_NAIVE || nrun == 0) {
    *admit = 1;
    return CI_OK;
  }
  std::vector<const ci_profile_t*> group;
  for (int i = 0; i < nrun; ++i) {
    const ci_profile_t* pr = profile_of(p, running_kinds[i]);
    if (!pr) return set_err(CI_ERR_INVALID_ARG, "ci_admit: no profile for kind %d", running_kinds[i]);
    group.push_back(pr);
  }
  const ci_profile_t* cp = profile_of(p, cand_kind);
  if (!cp) return set_err(CI_ERR_INVALID_ARG, "ci_admit: no profile for kind %d", cand_kind);
  group.push_back(cp);
  if (p->kind == CI_POLICY_USHER) {
    double occ = p->background ? p->background->occ : 0.0;
    for (auto* g : group) occ += g->occ;
    *admit = occ < 1.0;
    return CI_OK;
  }
  for (size_t j = 0; j < group.size(); ++j)  // CI_POLICY_SENSITIVITY
    if (predict(group, j, p->background) > p->bound) return CI_OK;
  *admit = 1;
  return CI_OK;
}


namespace {

// Draw the request's inputs into the arena and launch it on `s`.
ci_status_t start_request(ci_ctx* ctx, const ci_request_t& q, uint8_t* base, hipStream_t s,
                          Running& run) {
  auto al = [](uint64_t b) { return (b + 255) & ~255ull; };
  ci_victim_desc_t& d = run.d;
  memset(&d, 0, sizeof(d));
  d.kind = q.kind;
  d.dtype = q.dtype;
  d.m = q.m;
  d.n = q.n;
  d.k = q.k;
  d.passes = 1;
  d.copies = 1;
  d.scale_a = d.scale_b = 1.0f;
  uint8_t* p = base;
  switch (q.kind) {
    case CI_VICTIM_TRIAD_F32: {
      float* b = (float*)p;
      float* c = (float*)(p + al(q.n * 4));
      float* a = (float*)(p + 2 * al(q.n * 4));
      HIPCHK(launch_fill_uniform(b, q.n, q.seed, s));
      HIPCHK(launch_fill_uniform(c, q.n, q.seed + 1, s));
      d.a = b;
      d.b = c;
      d.out = a;
      break;
    }
    case CI_VICTIM_GEMM: {
      const uint64_t e = elem_bytes(q.dtype);
      uint8_t* A = p;
      uint8_t* B = A + al(q.m * q.k * e);
      float* C = (float*)(B + al(q.n * q.k * e));
      float* stage = (float*)((uint8_t*)C + al(q.m * q.n * 4));
      if (q.dtype == CI_DT_F32) {
        HIPCHK(launch_fill_uniform((float*)A, q.m * q.k, q.seed, s));
        HIPCHK(launch_fill_uniform((float*)B, q.n * q.k, q.seed + 1, s));
      } else if (q.dtype == CI_DT_BF16) {
        HIPCHK(launch_fill_uniform(stage, q.m * q.k, q.seed, s));
        HIPCHK(launch_to_bf16(stage, q.m * q.k, (uint16_t*)A, s));
        HIPCHK(launch_fill_uniform(stage, q.n * q.k, q.seed + 1, s));
        HIPCHK(launch_to_bf16(stage, q.n * q.k, (uint16_t*)B, s));
      } else {
        return set_err(CI_ERR_UNSUPPORTED, "serve: FP8 GEMM requests are not served");
      }
      d.a = A;
      d.b = B;
      d.out = C;
      break;
    }
    case CI_VICTIM_GEMV: {
      uint16_t* W = (uint16_t*)p;
      uint16_t* x = (uint16_t*)(p + al(q.n * q.k * 2));
      float* y = (float*)((uint8_t*)x + al(q.k * 2));
      float* stage = (float*)((uint8_t*)y + al(q.n * 4));
      HIPCHK(launch_fill_uniform(stage, q.n * q.k, q.seed, s));
      HIPCHK(launch_to_bf16(stage, q.n * q.k, W, s));
      HIPCHK(launch_fill_uniform(stage, q.k, q.seed + 1, s));
      HIPCHK(launch_to_bf16(stage, q.k, x, s));
      d.a = W;
      d.b = x;
      d.out = y;
      break;
    }
    default: return set_err(CI_ERR_INVALID_ARG, "serve: request kind %d", q.kind);
  }
  ci_status_t st = launch_victim(ctx, &d, s, run.ev0, run.ev1);
  if (st != CI_OK) return st;
  HIPCHK(hipEventRecord(run.done, s));
  return CI_OK;
}

}  // namespace

namespace {

// The stressor serve_run_background holds for the whole run.
struct Background {
  ci_resource_t r;
  float intensity;
  const ci_stressor_opts_t* opts;
  void* ws;
  size_t ws_bytes;
  ci_stressor_report_t* rep;
};

// Queue check of the slot streams against the background stressor's queue.
// Two hardware queues can slow each other's kernels although they share no
// CU and no traffic (the pairwise effect the measurement calls check before
// colocating, see check_queue_pair): before the stressor starts, each slot
// runs a probe triad alone and beside an idle kernel on the stressor's CUs
// and queue, in counterbalanced order; a slot slowed by more than
// kSlotQueueTol gets a new stream, kSlotQueueAttempts times at most.  The
// new stream carries a mask of every CU: the runtime deals plain streams
// over a small pool of hardware queues (a new plain stream may land on the
// very queue it replaces), but gives each CU-masked stream a queue of its
// own, created while the old one exists.  If a slot stays slowed, the
// stressor's queue is replaced once and every slot checked again.  The
// context's queue counters (ci_queue_stats) count the checks.
constexpr double kSlotQueueTol = 1.05;
constexpr int kSlotQueueAttempts = 6;
constexpr int kSlotQueuePairs = 6;
constexpr uint64_t kProbeMaxElems = 1ull << 24;
constexpr uint64_t kProbeMinElems = 1ull << 20;

ci_status_t probe_ns(ci_ctx* ctx, const ci_victim_desc_t& d, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                     double* ns) {
  const ci_status_t st = launch_victim(ctx, &d, s, e0, e1);
  if (st != CI_OK) return st;
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.0f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  *ns = (double)ms * 1e6;
  return CI_OK;
}

ci_status_t check_slot_queues(ci_ctx* ctx, const Background& bg, std::vector<hipStream_t>& streams,
                              uint8_t* arena, uint64_t arena_bytes, hipEvent_t e0, hipEvent_t e1) {
  const int k = cus_for(ctx, bg.intensity);
  uint64_t n = std::min(kProbeMaxElems, arena_bytes / 12 / 64 * 64);
  if (k == 0 || n < kProbeMinElems) return CI_OK;  // nothing to pair, or no room for a probe
  ci_stressor_opts_t o{};
  o.threads = 256;  // one 256-thread work-group per stressed CU, 1 KiB of LDS, sleeping
  o.wg_per_cu = 1;
  o.knob = 1;
  o.deadline_ms = 1000;
  size_t need = 0;
  ci_status_t st = ci_workspace_size(CI_RES_OCCUPANCY, bg.intensity, &o, &need);
  if (st != CI_OK) return st;
  if (!bg.ws || bg.ws_bytes < need) return CI_OK;  // no room for the idle kernel
  float* b = (float*)arena;
  float* c = b + n;
  float* a = c + n;
  HIPCHK(launch_fill_uniform(b, n, 0x5EED0001ull, streams[0]));
  HIPCHK(launch_fill_uniform(c, n, 0x5EED0002ull, streams[0]));
  HIPCHK(hipStreamSynchronize(streams[0]));
  ci_victim_desc_t d{};
  d.kind = CI_VICTIM_TRIAD_F32;
  d.dtype = CI_DT_F32;
  d.n = n;
  d.passes = 1;
  d.copies = 1;
  d.scale_a = d.scale_b = 1.0f;
  d.a = b;
  d.b = c;
  d.out = a;
  uint32_t mask[8], all[8];
  mask_for(ctx, k, 0, mask);
  mask_for(ctx, cus_for(ctx, 1.0), 0, all);
  for (int round = 0; round < 2; ++round) {
    bool all_ok = true;
    for (size_t s = 0; s < streams.size(); ++s) {
      ++ctx->queue_checks;
      for (int attempt = 0;; ++attempt) {
        double t = 0.0;
        for (int w = 0; w < 2; ++w)
          if ((st = probe_ns(ctx, d, streams[s], e0, e1, &t)) != CI_OK) return st;
        std::vector<double> ta, ti;
        for (int r = 0; r < kSlotQueuePairs; ++r) {
          const bool idle_first = r & 1;
          double t_alone = 0.0, t_idle = 0.0;
          if (!idle_first && (st = probe_ns(ctx, d, streams[s], e0, e1, &t_alone)) != CI_OK) return st;
          ci_stressor_t* h = nullptr;
          if ((st = stressor_launch(ctx, CI_RES_OCCUPANCY, bg.intensity, streams[s], &o, bg.ws, bg.ws_bytes,
                                    &h)) != CI_OK)
            return st;
          const ci_status_t vst = probe_ns(ctx, d, streams[s], e0, e1, &t_idle);
          st = stressor_stop(h, nullptr);
          if (vst != CI_OK) return vst;
          if (st != CI_OK) return st;
          if (idle_first && (st = probe_ns(ctx, d, streams[s], e0, e1, &t_alone)) != CI_OK) return st;
          ta.push_back(t_alone);
          ti.push_back(t_idle);
        }
        if (median(ti) <= kSlotQueueTol * median(ta)) break;
        if (attempt + 1 >= kSlotQueueAttempts) {
          all_ok = false;
          if (round == 1) ++ctx->queue_unresolved;
          break;
        }
        ++ctx->queue_replaced;
        hipStream_t ns = nullptr;
        HIPCHK(hipExtStreamCreateWithCUMask(&ns, 8, all));
        (void)hipStreamSynchronize(streams[s]);
        (void)hipStreamDestroy(streams[s]);
        streams[s] = ns;
      }
    }
    if (all_ok) break;
    if (round == 0) {
      ++ctx->queue_replaced;
      if (!replace_masked_stream(ctx, mask)) return set_err(CI_ERR_HIP, "hipExtStreamCreateWithCUMask failed");
    }
  }
  return CI_OK;
}

ci_status_t serve_impl(ci_ctx_t* ctx, const ci_request_t* trace, int n, const ci_policy_t* p,
                       const Background* bg, ci_served_t* out) {
  if (!ctx || !p || n < 0 || (n && (!trace || !out)))
    return set_err(CI_ERR_INVALID_ARG, "serve_run: bad argument");
  if (p->slots < 1 || p->slots > 8) return set_err(CI_ERR_INVALID_ARG, "serve_run: slots must be in [1, 8]");
  if (p->hbm_budget < 4096) return set_err(CI_ERR_INVALID_ARG, "serve_run: HBM budget too small");
  for (int i = 0; i < n; ++i) {
    const ci_request_t& q = trace[i];
    if (i && q.arrival_s < trace[i - 1].arrival_s)
      return set_err(CI_ERR_INVALID_ARG, "serve_run: trace not sorted by arrival");
    if (q.kind == CI_VICTIM_GEMM && (q.dtype != CI_DT_BF16 && q.dtype != CI_DT_F32))
      return set_err(CI_ERR_INVALID_ARG, "serve_run: request %d dtype", i);
    if (q.kind == CI_VICTIM_GEMM && ((q.k * elem_bytes(q.dtype)) % 16 || !q.m || !q.n || !q.k))
      return set_err(CI_ERR_INVALID_ARG, "serve_run: request %d GEMM shape", i);
    if (q.kind == CI_VICTIM_GEMV && (q.k % 8 || !q.n || !q.k))
      return set_err(CI_ERR_INVALID_ARG, "serve_run: request %d GEMV shape", i);
    if (q.kind == CI_VICTIM_TRIAD_F32 && !q.n)
      return set_err(CI_ERR_INVALID_ARG, "serve_run: request %d empty triad", i);
    if (q.kind < 0 || q.kind > CI_VICTIM_GEMV) return set_err(CI_ERR_INVALID_ARG, "serve_run: request %d kind", i);
    if (footprint(q) > p->hbm_budget)
      return set_err(CI_ERR_OOM, "serve_run: request %d needs %llu bytes > budget", i,
                     (unsigned long long)footprint(q));
    if (p->kind != CI_POLICY_NAIVE && !profile_of(p, q.kind))
      return set_err(CI_ERR_INVALID_ARG, "serve_run: no profile for request %d kind %d", i, q.kind);
  }
  if (ctx->active) return set_err(CI_ERR_BUSY, "serve_run: a stressor is running");
  HIPCHK(hipSetDevice(ctx->device));
  uint8_t* arena_base = nullptr;
  HIPCHK(hipMalloc((void**)&arena_base, p->hbm_budget));
  // per-slot streams, events and checksum scratch
  const int S = p->slots;
  std::vector<hipStream_t> streams(S, nullptr);
  std::vector<Running> slot(S);
  uint64_t* part_bits = nullptr;
  double* part_sum = nullptr;
  uint64_t* res = nullptr;  // pinned: [slot][2]
  const uint32_t nparts = 256;
  ci_status_t st = CI_OK;
  auto fail = [&](ci_status_t s2) { if (st == CI_OK) st = s2; };
  if (hipMalloc((void**)&part_bits, (size_t)S * nparts * 8) != hipSuccess ||
      hipMalloc((void**)&part_sum, (size_t)S * nparts * 8) != hipSuccess ||
      hipHostMalloc((void**)&res, (size_t)S * 2 * 8, hipHostMallocCoherent) != hipSuccess)
    fail(set_err(CI_ERR_OOM, "serve_run: scratch"));
  for (int s = 0; s < S && st == CI_OK; ++s) {
    if (hipStreamCreateWithFlags(&streams[s], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&slot[s].ev0) != hipSuccess || hipEventCreate(&slot[s].ev1) != hipSuccess ||
        hipEventCreateWithFlags(&slot[s].done, hipEventDisableTiming) != hipSuccess)
      fail(set_err(CI_ERR_HIP, "serve_run: stream/event creation"));
  }
  Arena arena(p->hbm_budget);
  std::deque<int> queue;
  std::vector<int> run_kinds;
  int next_arrival = 0, done = 0;
  // The background stressor starts after every allocation above (nothing
  // below allocates or frees device memory while it runs) and before the
  // trace's clock.
  ci_stressor_t* bg_h = nullptr;
  if (bg && st == CI_OK) fail(check_slot_queues(ctx, *bg, streams, arena_base, p->hbm_budget, slot[0].ev0,
                                                slot[0].ev1));
  if (bg && st == CI_OK) {
    const ci_status_t ls = stressor_launch(ctx, bg->r, bg->intensity, streams[0], bg->opts, bg->ws,
                                           bg->ws_bytes, &bg_h);
    if (ls != CI_OK) fail(ls);
  }
  const double t0 = now_s();
  for (int i = 0; i < n; ++i) {
    memset(&out[i], 0, sizeof(out[i]));
    out[i].arrival_s = trace[i].arrival_s;
    out[i].slot = -1;
  }
  while (st == CI_OK && done < n) {
    const double t = now_s() - t0;
    while (next_arrival < n && trace[next_arrival].arrival_s <= t) queue.push_back(next_arrival++);
    bool progressed = false;
    // retire finished requests
    for (int s = 0; s < S; ++s) {
      Running& r = slot[s];
      if (r.idx < 0) continue;
      hipError_t q = hipEventQuery(r.done);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) {
        fail(set_err(CI_ERR_HIP, "serve_run: request %d: %s", r.idx, hipGetErrorString(q)));
        break;
      }
      ci_served_t& o = out[r.idx];
      o.end_s = now_s() - t0;
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, r.ev0, r.ev1);
      o.service_ns = (double)ms * 1e6;
      o.checksum_bits = res[2 * s];
      memcpy(&o.sum_f64, (const void*)&res[2 * s + 1], 8);
      o.status = CI_OK;
      arena.release(r.off, r.bytes);
      r.idx = -1;
      ++done;
      progressed = true;
    }
    if (st != CI_OK) break;
    // admit FIFO, no bypass
    while (!queue.empty()) {
      int s = -1;
      run_kinds.clear();
      for (int k = 0; k < S; ++k) {
        if (slot[k].idx < 0) { if (s < 0) s = k; }
        else run_kinds.push_back(trace[slot[k].idx].kind);
      }
      if (s < 0) break;
      const ci_request_t& q = trace[queue.front()];
      const uint64_t bytes = (footprint(q) + 255) & ~255ull;
      int ok = 0;
      ci_status_t a = ci_admit(p, run_kinds.data(), (int)run_kinds.size(), q.kind, bytes,
                               arena.largest_free(), &ok);
      if (a != CI_OK) { fail(a); break; }
      if (!ok) break;
      uint64_t off = 0;
      if (!arena.alloc(bytes, &off)) break;
      Running& r = slot[s];
      r.idx = queue.front();
      r.off = off;
      r.bytes = bytes;
      queue.pop_front();
      out[r.idx].admit_s = now_s() - t0;
      out[r.idx].slot = s;
      ci_status_t ls = start_request(ctx, q, arena_base + off, streams[s], r);
      if (ls == CI_OK) {
        const uint64_t out_len = q.kind == CI_VICTIM_GEMM ? q.m * q.n : q.n;
        hipError_t e = launch_checksum_f32((const float*)r.d.out, out_len,
                                           part_bits + (size_t)s * nparts, part_sum + (size_t)s * nparts,
                                           nparts, &res[2 * s], (double*)&res[2 * s + 1], streams[s]);
        if (e == hipSuccess && q.out_copy)
          e = hipMemcpyAsync(q.out_copy, r.d.out, out_len * sizeof(float), hipMemcpyDeviceToDevice,
                             streams[s]);
        if (e == hipSuccess) e = hipEventRecord(r.done, streams[s]);
        if (e != hipSuccess) ls = set_err(CI_ERR_HIP, "serve_run: checksum: %s", hipGetErrorString(e));
      }
      if (ls != CI_OK) { fail(ls); break; }
      progressed = true;
    }
    if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
  if (bg_h) {  // stop it first: requests still queued may need its CUs
    const std::string why = st == CI_OK ? std::string() : std::string(ci_last_error());
    const ci_status_t ss = stressor_stop(bg_h, bg->rep);
    if (st == CI_OK)
      st = ss;
    else
      set_err(st, "%s", why.c_str());
  }
  // drain whatever is still on the device before freeing
  for (int s = 0; s < S; ++s)
    if (streams[s]) (void)hipStreamSynchronize(streams[s]);
  for (int s = 0; s < S; ++s) {
    if (slot[s].ev0) (void)hipEventDestroy(slot[s].ev0);
    if (slot[s].ev1) (void)hipEventDestroy(slot[s].ev1);
    if (slot[s].done) (void)hipEventDestroy(slot[s].done);
    if (streams[s]) (void)hipStreamDestroy(streams[s]);
  }
  if (res) (void)hipHostFree(res);
  if (part_bits) (void)hipFree(part_bits);
  if (part_sum) (void)hipFree(part_sum);
  (void)hipFree(arena_base);
  return st;
}

}  // namespace

extern "C" ci_status_t serve_run(ci_ctx_t* ctx, const ci_request_t* trace, int n,
                                 const ci_policy_t* p, ci_served_t* out) {
  return serve_impl(ctx, trace, n, p, nullptr, out);
}

extern "C" ci_status_t serve_run_background(ci_ctx_t* ctx, const ci_request_t* trace, int n,
                                            const ci_policy_t* p, ci_resource_t resource,
                                            float intensity, const ci_stressor_opts_t* opts, void* ws,
                                            size_t ws_bytes, ci_served_t* out,
                                            ci_stressor_report_t* rep) {
  if (!opts || !rep) return set_err(CI_ERR_INVALID_ARG, "serve_run_background: NULL opts or report");
  if (opts->passes != 0)
    return set_err(CI_ERR_INVALID_ARG, "serve_run_background: the stressor must run until stopped (passes 0)");
  memset(rep, 0, sizeof(*rep));
  const Background bg{resource, intensity, opts, ws, ws_bytes, rep};
  return serve_impl(ctx, trace, n, p, &bg, out);
}
