// Internal declarations shared by the libcoloc translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

#include <tuple>
#include <utility>

#include "../../include/coloc.h"

namespace ci {

// ---------------------------------------------------------------------------
// Control words a persistent stressor polls.
//
// The host raises `stop` in pinned, host-coherent memory.  Only one wave (the
// first wave of work-group 0, "the poller") reads that word over the bus; when
// it sees it set it copies it into `dev_stop`, which lives in device memory
// and is what every other wave polls.  Each wave polls at most once per
// `check_ticks` of the device wall clock, and every wave also stops on its own
// deadline, so every wave exits even if the host never raises the flag.
// ---------------------------------------------------------------------------
struct HostCtrl {           // pinned host memory, one per context
  volatile uint32_t stop;
  volatile uint32_t started;
  uint32_t pad[14];
};

struct DevCtrl {            // first 256 bytes of a stressor workspace
  uint32_t dev_stop;        // set by the poller
  uint32_t started;         // work-groups that have begun
  uint32_t pad0[14];
  uint64_t dispatch_count;  // DISPATCH counting form
  uint64_t pad1[23];
};
static_assert(sizeof(DevCtrl) == 256, "DevCtrl must stay 256 bytes");

struct KCtrl {              // by-value kernel argument
  HostCtrl* host;           // NULL in fixed-pass mode
  DevCtrl* dev;
  ci_wg_record_t* rec;
  uint64_t deadline_ticks;
  uint64_t check_ticks;
  uint64_t announce_ticks;  // poller waits at most this long for the grid
  uint64_t passes;          // 0 = persistent
  uint32_t grid;
  uint32_t duty;            // percent active, 1..100
};

constexpr uint32_t kRecFlagDeadline = 1u;
constexpr uint32_t kRecFlagStop = 2u;

// ------------------------------------------------------------------ device
__device__ __forceinline__ uint64_t dev_now() { return (uint64_t)wall_clock64(); }

// Hardware location of the calling wave: CU id, shader array, shader engine
// from HW_ID; XCD from XCC_ID (see the encoding in coloc.h).
__device__ __forceinline__ uint32_t hw_location() {
  const uint32_t hw = __builtin_amdgcn_s_getreg((31u << 11) | (0u << 6) | 4u);   // HW_ID, 32 bits
  const uint32_t xcc = __builtin_amdgcn_s_getreg((3u << 11) | (0u << 6) | 20u);  // XCC_ID[3:0]
  const uint32_t cu = (hw >> 8) & 0xFu;
  const uint32_t sh = (hw >> 12) & 0x1u;
  const uint32_t se = (hw >> 13) & 0x3u;
  return cu | (sh << 4) | (se << 5) | ((xcc & 0xFu) << 8);
}

__device__ __forceinline__ uint32_t load_sys(const volatile uint32_t* p) {
  return __hip_atomic_load(const_cast<uint32_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void store_sys(volatile uint32_t* p, uint32_t v) {
  __hip_atomic_store(const_cast<uint32_t*>(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint32_t load_agent(const uint32_t* p) {
  return __hip_atomic_load(const_cast<uint32_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_agent(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Per-wave stop state.
struct StopState {
  uint64_t deadline;
  uint64_t next_check;
  uint32_t flags;
  bool poller;
};

// Called by thread 0 of every work-group at entry: stamps the start, counts
// the work-group in, and (poller only) waits until the whole grid is resident
// or 50 ms pass, then tells the host the stressor is running.
__device__ __forceinline__ void wg_begin(const KCtrl& c, uint64_t& t0) {
  t0 = dev_now();
  if (c.host == nullptr) return;
  __hip_atomic_fetch_add(&c.dev->started, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void poller_announce(const KCtrl& c, uint64_t t0) {
  if (c.host == nullptr) return;
  while (load_agent(&c.dev->started) < c.grid && dev_now() - t0 < c.announce_ticks) {
    __builtin_amdgcn_s_sleep(8);
  }
  store_sys(&c.host->started, 1u);
}

__device__ __forceinline__ void stop_init(StopState& s, const KCtrl& c, uint64_t t0, bool poller) {
  s.deadline = t0 + c.deadline_ticks;
  s.next_check = t0 + c.check_ticks;
  s.flags = 0;
  s.poller = poller;
}

// Wave-uniform: true when this wave must stop (persistent mode only).
__device__ __forceinline__ bool should_stop(StopState& s, const KCtrl& c) {
  const uint64_t now = dev_now();
  if (now >= s.deadline) { s.flags |= kRecFlagDeadline; return true; }
  if (now < s.next_check) return false;
  s.next_check = now + c.check_ticks;
  uint32_t v;
  if (s.poller) {
    v = load_sys(&c.host->stop);
    if (v) store_agent(&c.dev->dev_stop, 1u);
  } else {
    v = load_agent(&c.dev->dev_stop);
  }
  if (v) s.flags |= kRecFlagStop;
  return v != 0;
}

// Duty cycle (intensity along time instead of CUs).  A wave marks the start
// of a busy stretch; at each duty point it idles for (100/duty - 1) times the
// stretch it just worked, then marks again.  Duty points sit every few
// microseconds of work, so a victim sees the load interleaved finely rather
// than in long bursts.  With several stressor waves per SIMD the unit's load
// is not linear in duty (a wave that works while others idle runs faster), so
// callers take the measured rate, not duty, as the load.
__device__ __forceinline__ uint64_t duty_mark(const KCtrl& c) {
  return (c.duty >= 100u || c.duty == 0u) ? 0 : dev_now();
}
__device__ __forceinline__ void duty_point(const KCtrl& c, uint64_t& t_busy0) {
  if (c.duty >= 100u || c.duty == 0u) return;
  const uint64_t now = dev_now();
  const uint64_t until = now + (now - t_busy0) * (100u - c.duty) / c.duty;
  uint64_t t = now;
  while (t < until) {
    __builtin_amdgcn_s_sleep(2);
    t = dev_now();
  }
  t_busy0 = t;
}

__device__ __forceinline__ void write_record(const KCtrl& c, uint32_t wg, uint64_t t0,
                                             uint64_t work, uint64_t check, uint32_t flags) {
  ci_wg_record_t r;
  r.t_start = t0;
  r.work = work;
  r.check = check;
  r.loc = hw_location();
  r.flags = flags;
  r.pad = 0;
  r.t_end = dev_now();
  c.rec[wg] = r;
}

// Wave-wide sums (deterministic butterfly over the 64 lanes).
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// ------------------------------------------------------------ host launchers

template <typename Tup, size_t... I>
inline void fill_args(Tup& t, void** argv, std::index_sequence<I...>) {
  ((argv[I] = static_cast<void*>(&std::get<I>(t))), ...);
}

// Launch with optional start/stop events (kernel-exact timing); returns the
// runtime's status instead of discarding it.
template <typename... KArgs, typename... Args>
inline hipError_t xlaunch(void (*kernel)(KArgs...), dim3 grid, dim3 block, uint32_t shmem,
                          hipStream_t s, hipEvent_t e0, hipEvent_t e1, Args... args) {
  static_assert(sizeof...(KArgs) == sizeof...(Args), "kernel argument count");
  void* argv[sizeof...(Args) + 1];
  std::tuple<KArgs...> tup{static_cast<KArgs>(args)...};
  fill_args(tup, argv, std::index_sequence_for<KArgs...>{});
  if (!e0 && !e1)   // plain launch: capturable into a HIP graph
    return hipLaunchKernel(reinterpret_cast<const void*>(kernel), grid, block, argv, shmem, s);
  return hipExtLaunchKernel(reinterpret_cast<const void*>(kernel), grid, block, argv, shmem, s,
                            e0, e1, 0);
}
// Each returns hipSuccess or the launch error.  `grid` work-groups.
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_stamp(uint64_t* slot, hipStream_t s);
hipError_t launch_triad_stressor(const KCtrl& c, const float* b, const float* cc, float* a,
                                 uint64_t n, uint32_t threads, bool streaming, hipStream_t s,
                                 hipEvent_t e0, hipEvent_t e1);
hipError_t launch_triad_victim(const float* b, const float* c, float* a, uint64_t n,
                               uint32_t passes, uint32_t grid, hipStream_t s, hipEvent_t e0,
                               hipEvent_t e1);
hipError_t launch_cache_stressor(const KCtrl& c, const uint32_t* region, uint64_t region_words,
                                 uint64_t slice_words, uint32_t batch, uint32_t threads,
                                 hipStream_t s,
    hipEvent_t e0, hipEvent_t e1);
hipError_t launch_lds_stressor(const KCtrl& c, const uint32_t* window, uint32_t vw,
                               uint32_t stride, uint32_t threads, hipStream_t s,
    hipEvent_t e0, hipEvent_t e1);
hipError_t launch_valu_stressor(const KCtrl& c, float* out, uint32_t ilp, uint64_t iters,
                                float fa, float fb, uint32_t threads, hipStream_t s,
    hipEvent_t e0, hipEvent_t e1);
hipError_t launch_valu64_stressor(const KCtrl& c, double* out, uint32_t ilp, uint64_t iters,
                                  double fa, uint32_t threads, hipStream_t s, hipEvent_t e0,
                                  hipEvent_t e1);
hipError_t launch_mfma_stressor(const KCtrl& c, int dtype, const void* a, const void* b,
                                float* out, uint32_t accs, uint64_t iters, uint32_t threads,
                                hipStream_t s,
    hipEvent_t e0, hipEvent_t e1);
hipError_t launch_chase_stressor(const KCtrl& c, const uint32_t* next, uint64_t n, uint32_t* end,
                                 uint32_t chains, uint64_t hops, uint32_t threads, hipStream_t s,
    hipEvent_t e0, hipEvent_t e1);
hipError_t launch_dispatch_empty(uint32_t nwg, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
hipError_t launch_dispatch_count(uint32_t nwg, uint64_t* counter, hipStream_t s, hipEvent_t e0,
                                 hipEvent_t e1);
hipError_t launch_dispatch_announce(HostCtrl* host, hipStream_t s);
hipError_t launch_hog(const KCtrl& c, uint32_t lds_bytes, uint32_t threads, hipStream_t s,
    hipEvent_t e0, hipEvent_t e1);
hipError_t launch_probe(uint32_t nwg, uint32_t* out, hipStream_t s);
hipError_t launch_checksum_f32(const float* x, uint64_t n, uint64_t* part_bits, double* part_sum,
                               uint32_t nparts, uint64_t* out_bits, double* out_sum,
                               hipStream_t s);
hipError_t launch_amax_f32(const float* x, uint64_t n, float* part, uint32_t nparts, float* out,
                           hipStream_t s);
hipError_t launch_to_bf16(const float* x, uint64_t n, uint16_t* out, hipStream_t s);
hipError_t launch_to_fp8(const float* x, uint64_t n, const float* amax, uint8_t* out,
                         hipStream_t s);
hipError_t launch_gemm(int dtype, const void* a, const void* b, float* c, uint64_t m, uint64_t n,
                       uint64_t k, float scale, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
hipError_t launch_gemv_bf16(const uint16_t* w, const uint16_t* x, float* y, uint64_t n,
                            uint64_t k, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
hipError_t launch_fill_uniform(float* dst, uint64_t n, uint64_t seed, hipStream_t s);
// decode step
hipError_t launch_rmsnorm_bf16(const float* x, const uint16_t* g, uint16_t* y, uint32_t rows,
                               uint32_t n, float eps, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
// Fused decode GEMV (see k_decode.hip): out / h / (q_out, kc, vc) from rows
// of w times batch vectors, given as BF16 v or as FP32 x normalised with g.
struct GemvArgs {
  const uint16_t* w;
  const uint16_t* v;      // BF16 input: batch x k
  const float* x;         // normalised input: batch x k FP32, gain g, eps
  const uint16_t* g;
  const float* res;       // PLAIN: optional residual (may alias out)
  float* out;             // PLAIN: batch x rows FP32
  uint16_t* h;            // SILU: batch x rows/2 BF16
  const int32_t* pos;     // ROPE: device positions; q_out FP32, caches BF16
  float* q_out;
  uint16_t* kc;
  uint16_t* vc;
  uint32_t rows, k, batch;
  uint32_t nq, nkv, d, max_ctx;
  float eps, base;
};
constexpr int kEpiPlain = 0, kEpiSilu = 1, kEpiRope = 2;
hipError_t launch_gemv_fused(const GemvArgs& a, int input_norm, int epilogue, hipStream_t s,
                             hipEvent_t e0, hipEvent_t e1);
hipError_t launch_rope_append(const float* qkv, const int32_t* pos, float* q_out, uint16_t* kc,
                              uint16_t* vc, uint32_t batch, uint32_t nq, uint32_t nkv, uint32_t d,
                              uint32_t max_ctx, float base, hipStream_t s, hipEvent_t e0,
                              hipEvent_t e1);
hipError_t launch_attn_partial(const float* q, const uint16_t* kc, const uint16_t* vc,
                               const int32_t* pos, float* part, uint32_t batch, uint32_t nq,
                               uint32_t nkv, uint32_t d, uint32_t max_ctx, uint32_t nchunks,
                               uint32_t used_chunks, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
hipError_t launch_attn_combine(const float* part, const int32_t* pos, uint16_t* out, uint32_t batch,
                               uint32_t nq, uint32_t d, uint32_t nchunks, hipStream_t s, hipEvent_t e0,
                               hipEvent_t e1);
hipError_t launch_silu_mul(const float* gu, uint16_t* h, uint32_t f, uint32_t batch, hipStream_t s,
                           hipEvent_t e0, hipEvent_t e1);

// Victim constraints checked on the host before any launch.
constexpr uint32_t kTriadThreads = 256;
constexpr uint32_t kGemmTile = 128;

}  // namespace ci
