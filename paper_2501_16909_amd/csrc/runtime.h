// Host-side state of libcoloc (not part of the C ABI).
#pragma once

#include <array>
#include <atomic>
#include <map>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

struct ci_ctx {
  int device = 0;
  ci_device_info_t info{};
  ci::HostCtrl* host = nullptr;        // pinned: stop / started words
  volatile uint64_t* hres = nullptr;   // pinned: stamps and checksums written by kernels
  uint64_t* part_bits = nullptr;       // device scratch for reductions
  double* part_sum = nullptr;
  float* amax_part = nullptr;
  float* amax_out = nullptr;
  uint32_t* probe_buf = nullptr;
  uint32_t nparts = 0;
  std::map<std::array<uint32_t, 8>, hipStream_t> masked;  // CU-masked streams by mask
  std::map<std::array<uint32_t, 8>, uint64_t> masked_used; // last use (use_clock) per mask
  uint64_t use_clock = 0;
  // Streams a running measurement holds (its victim stream, by reference so
  // that a replacement is seen): never evicted from `masked`.
  std::vector<const hipStream_t*> held;
  // A stressor kernel that did not drain may still poll the stop word: the
  // context then refuses further stressor launches (CI_ERR_DRAIN).
  bool drain_failed = false;
  hipStream_t vstream = nullptr;       // non-blocking stream for shared-placement victims
  // Queue pairs that passed the queue-pair check (with the idle kernel's
  // shape) and victim streams kept after qualification, each valid only at
  // the queue generation it was verified in: every stream this library
  // creates or destroys starts a new generation, since the runtime may then
  // place the existing queues differently.
  struct QueuePair {
    hipStream_t victim, stressor;
    uint32_t threads, wg_per_cu;
    uint64_t gen;
    int unresolved;  // still above the tolerance after the last replacement
  };
  std::vector<QueuePair> queue_checked;
  std::vector<std::pair<hipStream_t, uint64_t>> queue_qualified;
  uint64_t queue_gen = 0;
  uint32_t queue_checks = 0, queue_replaced = 0, queue_unresolved = 0;
  hipEvent_t ev[12] = {};
  struct ci_stressor* active = nullptr;
  uint64_t rot = 0;                    // GEMV weight-copy rotation
  // decode step: positions staged host -> device, events per kernel launch
  int32_t* dec_pos_host = nullptr;     // pinned, kDecodeMaxBatch entries
  int32_t* dec_pos_dev = nullptr;
  std::vector<hipEvent_t> dec_ev;
  std::map<std::string, hipGraphExec_t> dec_graphs;   // captured decode steps
};

struct ci_stressor {
  ci_ctx* ctx = nullptr;
  ci_resource_t r = CI_RES_HBM;
  float intensity = 0.0f;
  int ncu = 0;
  uint32_t grid = 0;
  hipStream_t ms = nullptr;            // masked stream the kernel runs on
  hipStream_t caller = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  ci_stressor_opts_t o{};
  bool noop = false;
  bool persistent = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  std::thread feeder;                  // DISPATCH only
  std::atomic<int> feeder_stop{0};
  std::atomic<uint64_t> launched{0};
  hipError_t feeder_err = hipSuccess;
};

#define HIPCHK(call)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) return ci::set_err(CI_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

namespace ci {
constexpr size_t kMaxMaskedStreams = 8;
constexpr uint32_t kDecodeMaxBatch = 8;
constexpr size_t kDecodeMaxGraphs = 8;
double median(std::vector<double> v);
double quantile(std::vector<double> v, double q);
int cus_for(const ci_ctx* ctx, double intensity);
bool mask_covers_all_xcds(const ci_ctx* ctx, const uint32_t mask[8]);
ci_status_t set_err(ci_status_t st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
hipStream_t masked_stream(ci_ctx* ctx, const uint32_t mask[8]);
hipStream_t replace_masked_stream(ci_ctx* ctx, const uint32_t mask[8]);
// Queue-pair check before a colocated measurement: see runtime.hip.
// run(arg, s, &ns) runs the victim once alone on stream s and returns its
// time.  *vs may be replaced: vmask is the victim stream's CU mask, or NULL
// for the unmasked victim stream.  With a victim mask (disjoint CUs) the
// idle kernel takes the launch shape of stressor r with options so.
// *unresolved is set to 1 when the pair still interfered after the last
// replacement (the cell is then measured as placed).
ci_status_t check_queue_pair(ci_ctx* ctx, ci_resource_t r, const ci_stressor_opts_t* so,
                             float intensity, hipStream_t caller, hipStream_t* vs,
                             const uint32_t* vmask, void* ws, size_t ws_bytes,
                             ci_status_t (*run)(void*, hipStream_t, double*), void* arg,
                             int* unresolved);

// Marks a stream variable as held by the running measurement for the
// guard's lifetime: masked_stream() never evicts the stream it names.
struct HeldStream {
  ci_ctx* ctx;
  HeldStream(ci_ctx* c, const hipStream_t* s) : ctx(c) { ctx->held.push_back(s); }
  ~HeldStream() { ctx->held.pop_back(); }
  HeldStream(const HeldStream&) = delete;
  HeldStream& operator=(const HeldStream&) = delete;
};
void mask_for(const ci_ctx* ctx, int k, int complement, uint32_t mask[8]);
ci_status_t launch_victim(ci_ctx* ctx, const ci_victim_desc_t* d, hipStream_t s, hipEvent_t e0,
                          hipEvent_t e1);
ci_status_t run_victim(ci_ctx* ctx, const ci_victim_desc_t* d, hipStream_t caller, hipStream_t xs,
                       ci_victim_result_t* out);
// Fetches, once per device, the device address of the static scratch array
// that ci_attention_decode_noalloc works in; call with `device` current.
ci_status_t static_scratch_init(int device);
}  // namespace ci
