// Device-side control protocol and helpers shared by the stressor kernels:
// control blocks, stop polling, duty cycle, per-work-group records and wave
// reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

constexpr int kTicketSlots = 8;  // one work counter per XCD slot (work-group index mod 8)

struct DevCtrl {            // first kCtrlBytes bytes of a stressor workspace
  uint32_t dev_stop;        // set by the poller
  uint32_t started;         // work-groups that have begun
  uint32_t pad0[14];
  uint64_t dispatch_count;  // DISPATCH counting form
  uint64_t pad1[23];
  // streaming stressors: next ticket of each XCD slot, one 256-byte line
  // each so that no two slots share a cache line
  uint64_t ticket[kTicketSlots][32];
};
constexpr size_t kCtrlBytes = 2304;
static_assert(sizeof(DevCtrl) == kCtrlBytes, "DevCtrl layout");

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

}  // namespace ci
