// Memory-side kernels: the triad (bandwidth stressor and victim) and the
// cache working-set loop used for the vL1D, L2 and Infinity-Cache stressors.
//
// The paper's bandwidth microbenchmark is a copy kernel that keeps copying a
// large input array to an output array with vectorised loads (Section 3,
// Pitfall 2; Section 4.3, Table 1); its cache-pollution variant sweeps the
// per-instance data size to move the working set in and out of L2 (Section
// 4.3, Figure 3).  Here the default streaming form is the triad a = b + 3c
// (two FP32 input streams, one output stream); read-only, copy and
// write-only forms move the same arrays in other read/write proportions.
// The cache forms re-read a region sized to one level of the CDNA4
// hierarchy.
#include "internal.h"

namespace ci {
namespace {

__device__ __forceinline__ float triad1(float b, float c) {
  // two roundings: fl(b + fl(3c)); contraction into a fused multiply-add is
  // switched off for this expression
#pragma clang fp contract(off)
  const float t = 3.0f * c;
  return b + t;
}

__device__ __forceinline__ float4 triad4(float4 b, float4 c) {
  return make_float4(triad1(b.x, c.x), triad1(b.y, c.y), triad1(b.z, c.z), triad1(b.w, c.w));
}

typedef float vf4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ vf4 triad_v(vf4 b, vf4 c) {
  vf4 r;
  r.x = triad1(b.x, c.x);
  r.y = triad1(b.y, c.y);
  r.z = triad1(b.z, c.z);
  r.w = triad1(b.w, c.w);
  return r;
}

typedef uint32_t vu4 __attribute__((ext_vector_type(4)));

// Traffic mixes of the streaming stressor (the values are the public
// CI_HBM_* constants): bytes moved per element are 12, 8, 8 and 4.
enum HbmMix : uint32_t { kMixTriad = 1, kMixRead = 2, kMixCopy = 3, kMixWrite = 4 };

// Stored by the write-only mix: element i holds the bits of lo32(i) times an
// odd constant (so distinct i < 2^32 give distinct words).
constexpr uint32_t kWriteMul = 0x9E3779B1u;

template <bool NT, typename V>
__device__ __forceinline__ V ld(const V* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

template <bool NT, typename V>
__device__ __forceinline__ void st(V* p, V v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// One wave-chunk of 256 * U elements starting at `base`: U 16-byte accesses
// per lane and stream, all loads issued before the first store.  The
// read-only mix adds the 32-bit words it reads into `acc` (mod 2^32).
template <uint32_t MIX, bool NT, int U>
__device__ __forceinline__ void stream_chunk(const float* __restrict__ b, const float* __restrict__ c,
                                             float* __restrict__ a, uint64_t base, uint64_t n,
                                             uint32_t lane, uint32_t& acc) {
  constexpr uint64_t kCh = 256ull * U;
  if (base + kCh <= n) {
    if constexpr (MIX == kMixTriad) {
      const vf4* b4 = reinterpret_cast<const vf4*>(b + base);
      const vf4* c4 = reinterpret_cast<const vf4*>(c + base);
      vf4* a4 = reinterpret_cast<vf4*>(a + base);
      vf4 vb[U], vc[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        vb[u] = ld<NT>(b4 + u * 64 + lane);
        vc[u] = ld<NT>(c4 + u * 64 + lane);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) st<NT>(a4 + u * 64 + lane, triad_v(vb[u], vc[u]));
    } else if constexpr (MIX == kMixRead) {
      const vu4* b4 = reinterpret_cast<const vu4*>(b + base);
      const vu4* c4 = reinterpret_cast<const vu4*>(c + base);
      vu4 vb[U], vc[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        vb[u] = ld<NT>(b4 + u * 64 + lane);
        vc[u] = ld<NT>(c4 + u * 64 + lane);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const vu4 t = vb[u] + vc[u];
        acc += t.x + t.y + t.z + t.w;
      }
    } else if constexpr (MIX == kMixCopy) {
      const vu4* b4 = reinterpret_cast<const vu4*>(b + base);
      vu4* a4 = reinterpret_cast<vu4*>(a + base);
      vu4 vb[U];
#pragma unroll
      for (int u = 0; u < U; ++u) vb[u] = ld<NT>(b4 + u * 64 + lane);
#pragma unroll
      for (int u = 0; u < U; ++u) st<NT>(a4 + u * 64 + lane, vb[u]);
    } else {
      vu4* a4 = reinterpret_cast<vu4*>(a + base);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t i0 = (uint32_t)base + (uint32_t)(u * 256) + lane * 4u;
        const vu4 v = {i0 * kWriteMul, (i0 + 1u) * kWriteMul, (i0 + 2u) * kWriteMul,
                       (i0 + 3u) * kWriteMul};
        st<NT>(a4 + u * 64 + lane, v);
      }
    }
  } else {
    const uint32_t* bu = reinterpret_cast<const uint32_t*>(b);
    const uint32_t* cu = reinterpret_cast<const uint32_t*>(c);
    uint32_t* au = reinterpret_cast<uint32_t*>(a);
    for (uint64_t i = base + lane; i < n && i < base + kCh; i += 64) {
      if constexpr (MIX == kMixTriad) a[i] = triad1(b[i], c[i]);
      else if constexpr (MIX == kMixRead) acc += bu[i] + cu[i];
      else if constexpr (MIX == kMixCopy) au[i] = bu[i];
      else au[i] = (uint32_t)i * kWriteMul;
    }
  }
}

// Streaming stressor (HBM, and the Infinity Cache with a footprint that
// fits it).  The array's wave-chunks are split into eight contiguous
// ranges, one per XCD slot (work-group index mod 8: work-groups are dealt
// to the XCDs round-robin, so a slot is one XCD's work-groups); a slot's
// work-groups take the range in order, one round of one chunk per wave at a
// time, from a ticket counter of that slot (thread 0 fetches the next
// ticket while the round runs).  All active waves thus work on a narrow
// moving window of each range, as the waves of a large one-shot grid do,
// instead of drifting apart over the whole array as fixed per-wave strides
// do (a measured difference of 69 against 81 % of the HBM peak for the
// triad).  Fixed-pass mode hands out exactly `passes` sweeps of every range;
// persistent mode wraps around until stopped.  record.work counts the
// wave-chunks the work-group processed; for the read-only mix record.check
// is the sum of the words it read mod 2^32.
//
// A read-only stream to HBM is the exception: there fixed per-wave strides
// (wave w of W takes chunks w, w + W, ...; no tickets, no barriers) measured
// faster (90 against 77-83 % of the peak), so that form has its own kernel.
template <uint32_t MIX, bool NT, int U>
__global__ void __launch_bounds__(1024) strided_stressor(KCtrl c, const float* __restrict__ b,
                                                         const float* __restrict__ cc,
                                                         float* __restrict__ a, uint64_t n) {
  __shared__ uint64_t s_t0;
  __shared__ uint64_t s_work[16];
  __shared__ uint32_t s_flags[16];
  __shared__ uint32_t s_acc[16];
  const uint32_t lane = threadIdx.x & 63u, wid = threadIdx.x >> 6;
  const uint32_t wpg = blockDim.x >> 6;
  if (threadIdx.x == 0) {
    uint64_t t0;
    wg_begin(c, t0);
    s_t0 = t0;
    if (blockIdx.x == 0) poller_announce(c, t0);
  }
  __syncthreads();
  const uint64_t t0 = s_t0;
  constexpr uint64_t kCh = 256ull * U;
  const uint64_t gw = (uint64_t)blockIdx.x * wpg + wid;
  const uint64_t nw = (uint64_t)gridDim.x * wpg;
  const uint64_t nch = (n + kCh - 1) / kCh;
  uint64_t done = 0;
  uint32_t acc = 0;
  StopState sst;
  stop_init(sst, c, t0, blockIdx.x == 0 && wid == 0);
  uint64_t tp = duty_mark(c);
  if (c.passes) {
    for (uint64_t p = 0; p < c.passes; ++p)
      for (uint64_t ch = gw; ch < nch; ch += nw) {
        stream_chunk<MIX, NT, U>(b, cc, a, ch * kCh, n, lane, acc);
        duty_point(c, tp);
        ++done;
      }
  } else if (gw < nch) {
    uint64_t ch = gw;
    for (;;) {
      stream_chunk<MIX, NT, U>(b, cc, a, ch * kCh, n, lane, acc);
      duty_point(c, tp);
      ++done;
      ch += nw;
      if (ch >= nch) ch = gw;
      if (should_stop(sst, c)) break;
    }
  } else {
    while (!should_stop(sst, c)) __builtin_amdgcn_s_sleep(32);
  }
  const uint32_t wacc = wave_sum_u32(acc);
  if (lane == 0) {
    s_work[wid] = done;
    s_flags[wid] = sst.flags;
    s_acc[wid] = wacc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t w = 0;
    uint32_t f = 0, sum = 0;
    for (uint32_t i = 0; i < wpg; ++i) {
      w += s_work[i];
      f |= s_flags[i];
      sum += s_acc[i];
    }
    write_record(c, blockIdx.x, t0, w, sum, f);
  }
}

//
// FIXED (c.passes > 0) and persistent launches are separate instantiations,
// so that traces and counters tell the fixed-work launches apart.  At most
// 64 registers per wave: two stressor waves per SIMD (its default shape)
// then leave 384 of the SIMD's 512 for a victim, which is what the GEMM
// victim's two 187-register waves take.
template <uint32_t MIX, bool NT, int U, bool FIXED>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8)))
stream_stressor(KCtrl c, const float* __restrict__ b,
                                                        const float* __restrict__ cc,
                                                        float* __restrict__ a, uint64_t n) {
  __shared__ uint64_t s_t0;
  __shared__ uint64_t s_ticket;
  __shared__ uint32_t s_stop;
  __shared__ uint64_t s_work[16];
  __shared__ uint32_t s_acc[16];
  const uint32_t lane = threadIdx.x & 63u, wid = threadIdx.x >> 6;
  const uint32_t wpg = blockDim.x >> 6;
  const uint32_t nslots = gridDim.x >= (uint32_t)kTicketSlots ? (uint32_t)kTicketSlots : 1u;
  const uint32_t slot = blockIdx.x % nslots;
  uint64_t* ticket = &c.dev->ticket[slot][0];
  StopState sst;
  uint64_t nxt = 0;
  if (threadIdx.x == 0) {
    uint64_t t0;
    wg_begin(c, t0);
    s_t0 = t0;
    s_stop = 0;
    if (blockIdx.x == 0) poller_announce(c, t0);
    s_ticket = __hip_atomic_fetch_add(ticket, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    nxt = __hip_atomic_fetch_add(ticket, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  const uint64_t t0 = s_t0;
  stop_init(sst, c, t0, blockIdx.x == 0 && threadIdx.x == 0);
  constexpr uint64_t kCh = 256ull * U;
  const uint64_t nch = (n + kCh - 1) / kCh;
  const uint64_t lo = nch * slot / nslots, hi = nch * (slot + 1) / nslots;
  const uint64_t rounds = (hi - lo + wpg - 1) / wpg;  // tickets per sweep of the range
  const uint64_t total = FIXED ? c.passes * rounds : 0;
  uint64_t done = 0;
  uint32_t acc = 0;
  uint64_t tp = duty_mark(c);
  if (rounds) {
    for (;;) {
      const uint64_t t = s_ticket;
      if (FIXED && t >= total) break;
      const uint64_t ch = lo + (t % rounds) * wpg + wid;
      if (ch < hi) {
        stream_chunk<MIX, NT, U>(b, cc, a, ch * kCh, n, lane, acc);
        ++done;
      }
      duty_point(c, tp);
      __syncthreads();  // every wave has read s_ticket
      if (threadIdx.x == 0) {
        s_ticket = nxt;
        nxt = __hip_atomic_fetch_add(ticket, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (!FIXED && should_stop(sst, c)) s_stop = 1;
      }
      __syncthreads();
      if (!FIXED && s_stop) break;
      // the busy stretch restarts after the barriers: time spent waiting
      // there for the other waves' idle periods is not work, and counting it
      // would make each idle period a multiple of the previous one
      tp = duty_mark(c);
    }
  } else if (!FIXED) {  // an empty range: hold the slot until stopped
    for (;;) {
      if (threadIdx.x == 0 && should_stop(sst, c)) s_stop = 1;
      __syncthreads();
      if (s_stop) break;
      __builtin_amdgcn_s_sleep(32);
    }
  }
  const uint32_t wacc = wave_sum_u32(acc);
  if (lane == 0) {
    s_work[wid] = done;
    s_acc[wid] = wacc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t w = 0;
    uint32_t sum = 0;
    for (uint32_t i = 0; i < wpg; ++i) {
      w += s_work[i];
      sum += s_acc[i];
    }
    write_record(c, blockIdx.x, t0, w, sum, sst.flags);
  }
}

// Victim triad: one sweep of the whole array per launch (grid-stride over
// wave-chunks of 1024 elements); `passes` sweeps are `passes` launches, so
// that every sweep reads the whole array however many work-groups are
// resident (a loop over sweeps inside the kernel would let resident waves
// re-read their own chunks from the L2 while the others wait).
// With `passes` > 1 (the in-kernel form) every wave sweeps its own chunks
// that many times.
__global__ void __launch_bounds__(256) triad_victim(const float* __restrict__ b,
                                                    const float* __restrict__ c,
                                                    float* __restrict__ a, uint64_t n,
                                                    uint32_t passes) {
  constexpr uint64_t kChunk = 1024;
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t gw = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const uint64_t nw = (uint64_t)gridDim.x * (blockDim.x >> 6);
  const uint64_t nchunks = (n + kChunk - 1) / kChunk;
  for (uint32_t p = 0; p < passes; ++p)
  for (uint64_t ch = gw; ch < nchunks; ch += nw) {
    const uint64_t base = ch * kChunk;
    if (base + kChunk <= n) {
      const float4* b4 = reinterpret_cast<const float4*>(b + base);
      const float4* c4 = reinterpret_cast<const float4*>(c + base);
      float4* a4 = reinterpret_cast<float4*>(a + base);
      float4 vb[4], vc[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) { vb[u] = b4[u * 64 + lane]; vc[u] = c4[u * 64 + lane]; }
#pragma unroll
      for (int u = 0; u < 4; ++u) a4[u * 64 + lane] = triad4(vb[u], vc[u]);
    } else {
      for (uint64_t i = base + lane; i < n && i < base + kChunk; i += 64) a[i] = triad1(b[i], c[i]);
    }
  }
}

// Cache working-set loop.  Work-group g reads its span of `len` words once per
// pass: the whole region (slice_words == 0; each work-group starts at its own
// phase so that concurrent groups do not walk in lock-step) or its own slice
// [g * slice, (g + 1) * slice) mod region.  Threads read 16 bytes at a time,
// four loads in flight; every word of the span is read exactly once per pass.
// record.work = passes, record.check = sum of the words read, mod 2^32.
// Span length must be a multiple of 4 * blockDim.x words (checked on the host).
// Four loads per thread in flight: eight raise the L2 rate by 1-2 % of peak
// but also fill the CU's memory pipeline, so a victim sharing the CUs loses
// several times more to the pipeline than to the L2 itself.
__global__ void __launch_bounds__(1024) cache_stressor(KCtrl c, const uint32_t* __restrict__ region,
                                                       uint64_t region_words, uint64_t slice_words,
                                                       uint32_t batch) {
  __shared__ uint64_t s_t0;
  __shared__ uint32_t s_stop;
  __shared__ uint32_t s_part[16];
  const uint32_t lane = threadIdx.x & 63u, wid = threadIdx.x >> 6, wpg = blockDim.x >> 6;
  if (threadIdx.x == 0) {
    uint64_t t0;
    wg_begin(c, t0);
    s_t0 = t0;
    s_stop = 0;
    if (blockIdx.x == 0) poller_announce(c, t0);
  }
  __syncthreads();
  const uint64_t t0 = s_t0;
  const uint64_t len = slice_words ? slice_words : region_words;
  const uint64_t lo = slice_words ? ((uint64_t)blockIdx.x * slice_words) % region_words : 0;
  // One round = one 16-byte load per thread; the span is `rounds` rounds.
  // Counts fit 32 bits (checked on the host), so loop control stays scalar.
  const uint32_t rounds = (uint32_t)(len / (4ull * blockDim.x));
  const uint32_t phase = slice_words ? 0u : (uint32_t)(((uint64_t)blockIdx.x * 7u) % rounds);
  const uint4* base = reinterpret_cast<const uint4*>(region + lo) + threadIdx.x;
  const uint32_t stride = blockDim.x;
  StopState st;
  stop_init(st, c, t0, blockIdx.x == 0 && threadIdx.x == 0);
  uint32_t acc = 0;
  uint64_t passes = 0;
  uint64_t tp = duty_mark(c);
  for (;;) {
    for (uint32_t bt = 0; bt < batch; ++bt) {
      duty_point(c, tp);
      // rounds [phase, rounds) then [0, phase): each word once per pass
      for (int part = 0; part < 2; ++part) {
        uint32_t r = part ? 0u : phase;
        const uint32_t end = part ? phase : rounds;
        for (; r + 4 <= end; r += 4) {
          uint4 v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) v[u] = base[(uint64_t)(r + u) * stride];
#pragma unroll
          for (int u = 0; u < 4; ++u) acc += v[u].x + v[u].y + v[u].z + v[u].w;
        }
        for (; r < end; ++r) {
          const uint4 v = base[(uint64_t)r * stride];
          acc += v.x + v.y + v.z + v.w;
        }
      }
    }
    passes += batch;
    if (c.passes) {
      if (passes >= c.passes) break;
      continue;
    }
    if (threadIdx.x == 0 && should_stop(st, c)) s_stop = 1;
    __syncthreads();
    if (s_stop) break;
  }
  const uint32_t ws = wave_sum_u32(acc);
  if (lane == 0) s_part[wid] = ws;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tot = 0;
    for (uint32_t i = 0; i < wpg; ++i) tot += s_part[i];
    write_record(c, blockIdx.x, t0, passes, tot, st.flags);
  }
}

__global__ void zero_kernel(uint4* p, uint64_t n16, uint8_t* tail, uint32_t ntail) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    p[i] = make_uint4(0, 0, 0, 0);
  if (blockIdx.x == 0 && threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

__global__ void stamp_kernel(uint64_t* slot) {
  if (threadIdx.x == 0) *slot = dev_now();
}

}  // namespace

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  const uint64_t n16 = bytes / 16;
  const uint32_t ntail = (uint32_t)(bytes % 16);
  uint64_t g = (n16 + 255) / 256;
  if (g > 4096) g = 4096;
  if (g == 0) g = 1;
  return xlaunch(zero_kernel, dim3((uint32_t)g), dim3(256), 0, s, nullptr, nullptr, (uint4*)p, n16,
                 (uint8_t*)p + n16 * 16, ntail);
}

hipError_t launch_stamp(uint64_t* slot, hipStream_t s) {
  return xlaunch(stamp_kernel, dim3(1), dim3(64), 0, s, nullptr, nullptr, slot);
}

hipError_t launch_stream_stressor(const KCtrl& c, uint32_t mix, uint32_t chunk, const float* b,
                                  const float* cc, float* a, uint64_t n, uint32_t threads,
                                  bool streaming, bool strided, hipStream_t s, hipEvent_t e0,
                                  hipEvent_t e1) {
  const dim3 g(c.grid), t(threads);
  if (strided && mix == kMixRead) {
    switch (chunk) {
      case 1:
        return streaming ? xlaunch(strided_stressor<kMixRead, true, 1>, g, t, 0, s, e0, e1, c, b, cc, a, n)
                         : xlaunch(strided_stressor<kMixRead, false, 1>, g, t, 0, s, e0, e1, c, b, cc, a, n);
      case 2:
        return streaming ? xlaunch(strided_stressor<kMixRead, true, 2>, g, t, 0, s, e0, e1, c, b, cc, a, n)
                         : xlaunch(strided_stressor<kMixRead, false, 2>, g, t, 0, s, e0, e1, c, b, cc, a, n);
      default:
        return streaming ? xlaunch(strided_stressor<kMixRead, true, 4>, g, t, 0, s, e0, e1, c, b, cc, a, n)
                         : xlaunch(strided_stressor<kMixRead, false, 4>, g, t, 0, s, e0, e1, c, b, cc, a, n);
    }
  }
#define CI_STREAM_LAUNCH_F(M, U, F)                                                                \
  return streaming ? xlaunch(stream_stressor<M, true, U, F>, g, t, 0, s, e0, e1, c, b, cc, a, n)   \
                   : xlaunch(stream_stressor<M, false, U, F>, g, t, 0, s, e0, e1, c, b, cc, a, n)
#define CI_STREAM_LAUNCH(M, U)                   \
  if (c.passes) CI_STREAM_LAUNCH_F(M, U, true); \
  CI_STREAM_LAUNCH_F(M, U, false)
#define CI_STREAM_MIX(U)                              \
  switch (mix) {                                      \
    case kMixRead: CI_STREAM_LAUNCH(kMixRead, U);     \
    case kMixCopy: CI_STREAM_LAUNCH(kMixCopy, U);     \
    case kMixWrite: CI_STREAM_LAUNCH(kMixWrite, U);   \
    default: CI_STREAM_LAUNCH(kMixTriad, U);          \
  }
  switch (chunk) {
    case 1: CI_STREAM_MIX(1);
    case 4: CI_STREAM_MIX(4);
    default: CI_STREAM_MIX(2);
  }
#undef CI_STREAM_MIX
#undef CI_STREAM_LAUNCH
#undef CI_STREAM_LAUNCH_F
}

hipError_t launch_triad_victim(const float* b, const float* c, float* a, uint64_t n,
                               uint32_t passes, bool in_kernel, uint32_t grid, hipStream_t s,
                               hipEvent_t e0, hipEvent_t e1) {
  if (in_kernel)
    return xlaunch(triad_victim, dim3(grid), dim3(kTriadThreads), 0, s, e0, e1, b, c, a, n, passes);
  for (uint32_t p = 0; p < passes; ++p) {
    const hipError_t e = xlaunch(triad_victim, dim3(grid), dim3(kTriadThreads), 0, s, p == 0 ? e0 : nullptr,
                                 p + 1 == passes ? e1 : nullptr, b, c, a, n, 1u);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_cache_stressor(const KCtrl& c, const uint32_t* region, uint64_t region_words,
                                 uint64_t slice_words, uint32_t batch, uint32_t threads,
                                 hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  return xlaunch(cache_stressor, dim3(c.grid), dim3(threads), 0, s, e0, e1, c,
                               region, region_words, slice_words, batch);
}

}  // namespace ci
