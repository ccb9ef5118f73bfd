// On-CU stressors: LDS, VALU (FP32 FMA chains), matrix cores (MFMA), the
// pointer chase, work-group dispatch, the occupancy hog and the placement
// probe.
//
// Paper correspondences: the compute kernel (independent element-wise
// multiplies with an ILP knob, Section 3 Pitfall 1 and Sections 4.4.2-4.4.3)
// becomes FMA chains on the VALU and register-resident MFMA loops; the
// strided shared-memory copy (Section 4.4.1) becomes the LDS loop; the sleep
// kernel that holds SM resources and blocks the block scheduler (Section 4.2)
// becomes the occupancy hog; the per-block SM-ID print (Section 4.2
// footnote) becomes the placement probe.
#include <type_traits>

#include "internal.h"

namespace ci {
namespace {

// Work-group-uniform stop decision: thread 0 polls, the barrier publishes.
struct WgStop {
  StopState st;
  __device__ bool check(const KCtrl& c, uint32_t* s_stop) {
    if (threadIdx.x == 0 && should_stop(st, c)) *s_stop = 1;
    __syncthreads();
    return *s_stop != 0;
  }
};

__device__ __forceinline__ uint64_t wg_enter(const KCtrl& c, uint64_t* s_t0, uint32_t* s_stop) {
  if (threadIdx.x == 0) {
    uint64_t t0;
    wg_begin(c, t0);
    *s_t0 = t0;
    *s_stop = 0;
    if (blockIdx.x == 0) poller_announce(c, t0);
  }
  __syncthreads();
  return *s_t0;
}

// ------------------------------------------------------------------- LDS
// 64 KiB of LDS per work-group: two 32 KiB windows A and B holding the same
// 8192 words.  On each pass, lane l of every wave walks the window's
// nvec = 8192/VW vectors of VW words in the order (l*stride + k) mod nvec,
// reading each from one window and storing it to the same place in the
// other; the direction alternates every pass.  Stored values equal the ones
// already there, so the contents never change.  `stride` sets how many lanes
// of a wave land in the same bank.  LOAD: the same walk without the stores
// (the load path alone), reading each pass from A onward.  record.check =
// sum of words read mod 2^32.
template <int VW, bool LOAD>
__global__ void __launch_bounds__(1024) lds_stressor(KCtrl c, const uint32_t* __restrict__ window,
                                                     uint32_t stride) {
  extern __shared__ uint32_t lds[];
  __shared__ uint64_t s_t0;
  __shared__ uint32_t s_stop;
  __shared__ uint32_t s_part[16];
  constexpr uint32_t kWords = 8192, kVec = kWords / VW;
  const uint64_t t0 = wg_enter(c, &s_t0, &s_stop);
  for (uint32_t i = threadIdx.x; i < kWords; i += blockDim.x) {
    const uint32_t w = window[i];
    lds[i] = w;
    lds[kWords + i] = w;
  }
  __syncthreads();
  const uint32_t lane = threadIdx.x & 63u, wid = threadIdx.x >> 6, wpg = blockDim.x >> 6;
  const uint32_t v0 = (uint32_t)(((uint64_t)lane * stride) & (kVec - 1));
  WgStop ws;
  stop_init(ws.st, c, t0, blockIdx.x == 0 && threadIdx.x == 0);
  uint32_t acc = 0;
  uint64_t passes = 0;
  uint64_t tp = duty_mark(c);
  for (;;) {
    if constexpr (LOAD) {
      // Windows A and B are adjacent copies, so lane l's walk v0, v0+1, ...,
      // v0+kVec-1 (mod kVec) reads the same words straight through A into B:
      // no wrap, and the unrolled steps' addresses are immediate offsets.
      // The load path then runs with two 3-input adds per 16-byte load, and
      // the loads are issued in batches of 8 before their sums so that each
      // wave keeps several in flight.  The last word read is at
      // (2 kVec - 2) VW + VW - 1 < 2 kWords.
      using V = typename std::conditional<VW == 4, uint4, typename std::conditional<VW == 2, uint2, uint32_t>::type>::type;
      const V* base = reinterpret_cast<const V*>(lds + v0 * VW);
      for (uint32_t kg = 0; kg < kVec; kg += 256) {
        duty_point(c, tp);
        const V* p = base + kg;
        for (uint32_t k = 0; k < 256; k += 8) {
          V x[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) x[j] = p[k + j];
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            if constexpr (VW == 4) acc += x[j].x + x[j].y + x[j].z + x[j].w;
            else if constexpr (VW == 2) acc += x[j].x + x[j].y;
            else acc += x[j];
          }
        }
      }
    } else {
      uint32_t* src = (passes & 1) ? lds + kWords : lds;
      uint32_t* dst = (passes & 1) ? lds : lds + kWords;
      uint32_t v = v0;
      for (uint32_t kg = 0; kg < kVec; kg += 256) {
        duty_point(c, tp);
#pragma unroll 8
        for (uint32_t k = 0; k < 256; ++k) {
          if constexpr (VW == 4) {
            const uint4 x = *reinterpret_cast<const uint4*>(src + v * 4);
            *reinterpret_cast<uint4*>(dst + v * 4) = x;
            acc += x.x + x.y + x.z + x.w;
          } else if constexpr (VW == 2) {
            const uint2 x = *reinterpret_cast<const uint2*>(src + v * 2);
            *reinterpret_cast<uint2*>(dst + v * 2) = x;
            acc += x.x + x.y;
          } else {
            const uint32_t x = src[v];
            dst[v] = x;
            acc += x;
          }
          v = (v + 1) & (kVec - 1);
        }
      }
    }
    ++passes;
    if (c.passes) {
      if (passes >= c.passes) break;
      continue;
    }
    if (ws.check(c, &s_stop)) break;
  }
  const uint32_t t = wave_sum_u32(acc);
  __syncthreads();
  if (lane == 0) s_part[wid] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tot = 0;
    for (uint32_t i = 0; i < wpg; ++i) tot += s_part[i];
    write_record(c, blockIdx.x, t0, passes, tot, ws.st.flags);
  }
}

// ------------------------------------------------------------------ VALU
// ILP independent chains per lane, x <- fma(x, fa, fb), `iters` steps per
// pass.  Start value of chain j of global thread t: ((t mod 1024)+j+1)/1024.
// The chains continue across passes; dst[t*ILP + j] = final value.
template <int ILP>
__global__ void __launch_bounds__(1024) valu_stressor(KCtrl c, float* __restrict__ out, uint32_t iters,
                                                      float fa, float fb) {
  __shared__ uint64_t s_t0;
  __shared__ uint32_t s_stop;
  const uint64_t t0 = wg_enter(c, &s_t0, &s_stop);
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float x[ILP];
#pragma unroll
  for (int j = 0; j < ILP; ++j) x[j] = (float)((uint32_t)(t & 1023u) + j + 1) * 0x1.0p-10f;
  // An FMA may read only one scalar register: keep the addend in a vector
  // register for the whole loop (a lane broadcast of the same value).
  const float vb = __shfl(fb, 0, 64);
  WgStop ws;
  stop_init(ws.st, c, t0, blockIdx.x == 0 && threadIdx.x == 0);
  const uint32_t blocks = iters >> 3, rem = iters & 7u;
  uint64_t passes = 0;
  uint64_t tp = duty_mark(c);
  for (;;) {
    // groups of 64 blocks of 8 steps, a duty point after each group
    uint32_t blk = 0;
    for (; blk + 64 <= blocks; blk += 64) {
#pragma nounroll
      for (uint32_t g = 0; g < 64; ++g)
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int j = 0; j < ILP; ++j) x[j] = __builtin_fmaf(x[j], fa, vb);
      duty_point(c, tp);
    }
#pragma nounroll
    for (; blk < blocks; ++blk)
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int j = 0; j < ILP; ++j) x[j] = __builtin_fmaf(x[j], fa, vb);
    for (uint32_t r = 0; r < rem; ++r)
#pragma unroll
      for (int j = 0; j < ILP; ++j) x[j] = __builtin_fmaf(x[j], fa, vb);
    duty_point(c, tp);
    ++passes;
    if (c.passes) {
      if (passes >= c.passes) break;
      continue;
    }
    if (ws.check(c, &s_stop)) break;
  }
#pragma unroll
  for (int j = 0; j < ILP; ++j) out[t * ILP + j] = x[j];
  __syncthreads();
  if (threadIdx.x == 0) write_record(c, blockIdx.x, t0, passes, 0, ws.st.flags);
}

// ------------------------------------------------------------ VALU FP64
// The paper's FP64 pipeline kernel (Section 4.4.3): ILP independent chains of
// x <- x * a per lane, one rounded binary64 multiply per step; same start
// values and pass structure as the FP32 chains; dst[t*ILP + j] = final x.
template <int ILP>
__global__ void __launch_bounds__(1024) valu64_stressor(KCtrl c, double* __restrict__ out,
                                                        uint32_t iters, double fa) {
  __shared__ uint64_t s_t0;
  __shared__ uint32_t s_stop;
  const uint64_t t0 = wg_enter(c, &s_t0, &s_stop);
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double x[ILP];
#pragma unroll
  for (int j = 0; j < ILP; ++j) x[j] = (double)((uint32_t)(t & 1023u) + j + 1) * 0x1.0p-10;
  WgStop ws;
  stop_init(ws.st, c, t0, blockIdx.x == 0 && threadIdx.x == 0);
  const uint32_t blocks = iters >> 3, rem = iters & 7u;
  uint64_t passes = 0;
  uint64_t tp = duty_mark(c);
  for (;;) {
    // groups of 64 blocks of 8 steps, a duty point after each group
    uint32_t blk = 0;
    for (; blk + 64 <= blocks; blk += 64) {
#pragma nounroll
      for (uint32_t g = 0; g < 64; ++g)
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int j = 0; j < ILP; ++j) x[j] = __dmul_rn(x[j], fa);
      duty_point(c, tp);
    }
#pragma nounroll
    for (; blk < blocks; ++blk)
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int j = 0; j < ILP; ++j) x[j] = __dmul_rn(x[j], fa);
    for (uint32_t r = 0; r < rem; ++r)
#pragma unroll
      for (int j = 0; j < ILP; ++j) x[j] = __dmul_rn(x[j], fa);
    duty_point(c, tp);
    ++passes;
    if (c.passes) {
      if (passes >= c.passes) break;
      continue;
    }
    if (ws.check(c, &s_stop)) break;
  }
#pragma unroll
  for (int j = 0; j < ILP; ++j) out[t * ILP + j] = x[j];
  __syncthreads();
  if (threadIdx.x == 0) write_record(c, blockIdx.x, t0, passes, 0, ws.st.flags);
}

// ------------------------------------------------------------------ MFMA
// Every wave keeps NACC accumulators of one 32x32 output tile and adds the
// same product A (32 x K) * B (K x 32) to each, `iters` times per pass, with
// no memory traffic inside the loop.  Operand layout of the 32x32xK
// instructions: lane l supplies row (l mod 32) of A and column (l mod 32) of
// B, for the K-block selected by l / 32; both operands use the same K order,
// so the product does not depend on how the hardware orders K inside a lane.
// Accumulator register v of lane l holds C[8*(v/4) + 4*(l/32) + v%4][l mod 32].
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

template <int DT>
struct MfmaOp;

template <>
struct MfmaOp<CI_DT_F32> {
  static constexpr int K = 2;
  typedef float frag;
  __device__ static frag load_a(const void* a, uint32_t lane) {
    return reinterpret_cast<const float*>(a)[(lane & 31u) * K + (lane >> 5)];
  }
  __device__ static frag load_b(const void* b, uint32_t lane) {
    return reinterpret_cast<const float*>(b)[(lane >> 5) * 32 + (lane & 31u)];
  }
  __device__ static f32x16 mma(frag a, frag b, f32x16 acc) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
  }
};

template <>
struct MfmaOp<CI_DT_BF16> {
  static constexpr int K = 16;
  typedef bf16x8 frag;
  __device__ static frag load_a(const void* a, uint32_t lane) {
    const __bf16* p = reinterpret_cast<const __bf16*>(a) + (lane & 31u) * K + (lane >> 5) * 8;
    frag f;
#pragma unroll
    for (int j = 0; j < 8; ++j) f[j] = p[j];
    return f;
  }
  __device__ static frag load_b(const void* b, uint32_t lane) {
    const __bf16* p = reinterpret_cast<const __bf16*>(b);
    frag f;
#pragma unroll
    for (int j = 0; j < 8; ++j) f[j] = p[((lane >> 5) * 8 + j) * 32 + (lane & 31u)];
    return f;
  }
  __device__ static f32x16 mma(frag a, frag b, f32x16 acc) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  }
};

template <>
struct MfmaOp<CI_DT_FP8E4M3> {
  static constexpr int K = 64;
  typedef i32x8 frag;  // 32 E4M3 bytes
  __device__ static frag load_a(const void* a, uint32_t lane) {
    const uint8_t* p = reinterpret_cast<const uint8_t*>(a) + (lane & 31u) * K + (lane >> 5) * 32;
    frag f;
#pragma unroll
    for (int j = 0; j < 8; ++j)
      f[j] = (int)((uint32_t)p[4 * j] | ((uint32_t)p[4 * j + 1] << 8) |
                   ((uint32_t)p[4 * j + 2] << 16) | ((uint32_t)p[4 * j + 3] << 24));
    return f;
  }
  __device__ static frag load_b(const void* b, uint32_t lane) {
    const uint8_t* p = reinterpret_cast<const uint8_t*>(b);
    frag f;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      uint32_t w = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) w |= (uint32_t)p[((lane >> 5) * 32 + 4 * j + q) * 32 + (lane & 31u)] << (8 * q);
      f[j] = (int)w;
    }
    return f;
  }
  __device__ static f32x16 mma(frag a, frag b, f32x16 acc) {
    // format selectors 0/0 = E4M3 for both operands; zero scales select the
    // unscaled instruction
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, acc, 0, 0, 0, 0, 0, 0);
  }
};

template <int DT, int NACC>
__global__ void __launch_bounds__(1024) mfma_stressor(KCtrl c, const void* __restrict__ a,
                                                      const void* __restrict__ b,
                                                      float* __restrict__ out, uint64_t iters) {
  using Op = MfmaOp<DT>;
  __shared__ uint64_t s_t0;
  __shared__ uint32_t s_stop;
  const uint64_t t0 = wg_enter(c, &s_t0, &s_stop);
  const uint32_t lane = threadIdx.x & 63u;
  const typename Op::frag fa = Op::load_a(a, lane);
  const typename Op::frag fb = Op::load_b(b, lane);
  f32x16 acc[NACC];
#pragma unroll
  for (int q = 0; q < NACC; ++q)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[q][v] = 0.0f;
  WgStop ws;
  stop_init(ws.st, c, t0, blockIdx.x == 0 && threadIdx.x == 0);
  uint64_t passes = 0;
  uint64_t tp = duty_mark(c);
  for (;;) {
    // groups of 32 steps, a duty point after each group
    uint64_t it = 0;
    for (; it + 32 <= iters; it += 32) {
      for (int g = 0; g < 32; ++g)
#pragma unroll
        for (int q = 0; q < NACC; ++q) acc[q] = Op::mma(fa, fb, acc[q]);
      duty_point(c, tp);
    }
    for (; it < iters; ++it)
#pragma unroll
      for (int q = 0; q < NACC; ++q) acc[q] = Op::mma(fa, fb, acc[q]);
    duty_point(c, tp);
    ++passes;
    if (c.passes) {
      if (passes >= c.passes) break;
      continue;
    }
    if (ws.check(c, &s_stop)) break;
  }
  const uint64_t gwave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
#pragma unroll
  for (int q = 0; q < NACC; ++q) {
    float* tile = out + (gwave * NACC + q) * 1024;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const uint32_t row = 8u * (v / 4) + 4u * (lane >> 5) + (v % 4);
      tile[row * 32 + (lane & 31u)] = acc[q][v];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) write_record(c, blockIdx.x, t0, passes, 0, ws.st.flags);
}

// One matrix-core instruction per tile: D = A B + C, with A, B and the
// accumulator input C loaded in the stressor's fragment layout (A 32 x K and
// B K x 32 row-major, K = 2 / 16 / 64 for FP32 / BF16 / E4M3; C and D 32 x 32
// FP32 row-major).  Tile t is work-group t (one wave).
template <int DT>
__global__ void __launch_bounds__(64) mfma_probe_kernel(const uint8_t* __restrict__ a,
                                                        const uint8_t* __restrict__ b,
                                                        const float* __restrict__ c,
                                                        float* __restrict__ d) {
  using Op = MfmaOp<DT>;
  constexpr uint32_t kOpBytes = 32u * Op::K * (DT == CI_DT_F32 ? 4u : DT == CI_DT_BF16 ? 2u : 1u);
  const uint32_t lane = threadIdx.x;
  const size_t t = blockIdx.x;
  const typename Op::frag fa = Op::load_a(a + t * kOpBytes, lane);
  const typename Op::frag fb = Op::load_b(b + t * kOpBytes, lane);
  const float* ct = c + t * 1024;
  float* dt = d + t * 1024;
  f32x16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = ct[(8u * (v / 4) + 4u * (lane >> 5) + (v % 4)) * 32 + (lane & 31u)];
  acc = Op::mma(fa, fb, acc);
#pragma unroll
  for (int v = 0; v < 16; ++v) dt[(8u * (v / 4) + 4u * (lane >> 5) + (v % 4)) * 32 + (lane & 31u)] = acc[v];
}

// --------------------------------------------------------- pointer chase
// CH independent chains per lane; global chain q of Q starts at floor(q*n/Q)
// and follows next[] `hops` times per pass; dst[q] = index reached.  Table
// entries >= n are read as n - 1 (never reached with a valid permutation).
template <int CH>
__global__ void __launch_bounds__(1024) chase_stressor(KCtrl c, const uint32_t* __restrict__ next,
                                                       uint64_t n, uint32_t* __restrict__ end,
                                                       uint64_t hops) {
  __shared__ uint64_t s_t0;
  __shared__ uint32_t s_stop;
  const uint64_t t0 = wg_enter(c, &s_t0, &s_stop);
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t nq = (uint64_t)gridDim.x * blockDim.x * CH;
  const uint32_t nmax = (uint32_t)(n - 1);
  uint32_t idx[CH];
#pragma unroll
  for (int j = 0; j < CH; ++j) {
    const uint64_t q = t * CH + j;
    idx[j] = (uint32_t)(q * n / nq);  // q < 2^31, n <= 2^32: no overflow
  }
  WgStop ws;
  stop_init(ws.st, c, t0, blockIdx.x == 0 && threadIdx.x == 0);
  uint64_t passes = 0;
  uint64_t tp = duty_mark(c);
  for (;;) {
    for (uint64_t h = 0; h < hops; ++h) {
      if ((h & 15u) == 15u) duty_point(c, tp);
#pragma unroll
      for (int j = 0; j < CH; ++j) idx[j] = min(next[idx[j]], nmax);  // clamp: a bad table cannot read out of bounds
    }
    duty_point(c, tp);
    ++passes;
    if (c.passes) {
      if (passes >= c.passes) break;
      continue;
    }
    if (ws.check(c, &s_stop)) break;
  }
#pragma unroll
  for (int j = 0; j < CH; ++j) end[t * CH + j] = idx[j];
  __syncthreads();
  if (threadIdx.x == 0) write_record(c, blockIdx.x, t0, passes, 0, ws.st.flags);
}

// -------------------------------------------------------------- dispatch
__global__ void __launch_bounds__(64) empty_wg() {}

__global__ void __launch_bounds__(64) count_wg(uint64_t* counter) {
  if (threadIdx.x == 0)
    __hip_atomic_fetch_add(counter, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void announce_wg(HostCtrl* host) {
  if (threadIdx.x == 0) store_sys(&host->started, 1u);
}

// --------------------------------------------------------- occupancy hog
// Holds `lds_bytes` of LDS and its wave slots while sleeping; never touches
// memory beyond its record.  record.work = sleep rounds.
__global__ void __launch_bounds__(1024) hog_kernel(KCtrl c, uint32_t lds_words) {
  extern __shared__ uint32_t lds[];
  __shared__ uint64_t s_t0;
  __shared__ uint32_t s_stop;
  const uint64_t t0 = wg_enter(c, &s_t0, &s_stop);
  for (uint32_t i = threadIdx.x; i < lds_words; i += blockDim.x) lds[i] = i;
  WgStop ws;
  stop_init(ws.st, c, t0, blockIdx.x == 0 && threadIdx.x == 0);
  uint64_t rounds = 0;
  for (;;) {
    __builtin_amdgcn_s_sleep(127);
    ++rounds;
    if (c.passes) {
      if (rounds >= c.passes) break;
      __syncthreads();
      continue;
    }
    if (ws.check(c, &s_stop)) break;
  }
  __syncthreads();
  if (threadIdx.x == 0) write_record(c, blockIdx.x, t0, rounds, lds_words ? lds[lds_words - 1] : 0, ws.st.flags);
}

// ------------------------------------------------------- placement probe
__global__ void __launch_bounds__(64) probe_kernel(uint32_t* out) {
  if (threadIdx.x == 0) out[blockIdx.x] = hw_location();
}

}  // namespace

hipError_t launch_lds_stressor(const KCtrl& c, const uint32_t* window, uint32_t vw, uint32_t stride,
                               bool load_only, uint32_t threads, hipStream_t s, hipEvent_t e0,
                               hipEvent_t e1) {
  const uint32_t shm = 2 * 8192 * 4;
  const dim3 g(c.grid), t(threads);
  if (load_only) {
    switch (vw) {
      case 1: return xlaunch(lds_stressor<1, true>, g, t, shm, s, e0, e1, c, window, stride);
      case 2: return xlaunch(lds_stressor<2, true>, g, t, shm, s, e0, e1, c, window, stride);
      default: return xlaunch(lds_stressor<4, true>, g, t, shm, s, e0, e1, c, window, stride);
    }
  }
  switch (vw) {
    case 1: return xlaunch(lds_stressor<1, false>, g, t, shm, s, e0, e1, c, window, stride);
    case 2: return xlaunch(lds_stressor<2, false>, g, t, shm, s, e0, e1, c, window, stride);
    default: return xlaunch(lds_stressor<4, false>, g, t, shm, s, e0, e1, c, window, stride);
  }
}

hipError_t launch_valu_stressor(const KCtrl& c, float* out, uint32_t ilp, uint64_t iters64, float fa,
                                float fb, uint32_t threads, hipStream_t s, hipEvent_t e0,
                                hipEvent_t e1) {
  const uint32_t iters = (uint32_t)iters64;  // range checked by the caller
  switch (ilp) {
    case 1: return xlaunch(valu_stressor<1>, dim3(c.grid), dim3(threads), 0, s, e0, e1, c, out, iters, fa, fb);
    case 2: return xlaunch(valu_stressor<2>, dim3(c.grid), dim3(threads), 0, s, e0, e1, c, out, iters, fa, fb);
    case 4: return xlaunch(valu_stressor<4>, dim3(c.grid), dim3(threads), 0, s, e0, e1, c, out, iters, fa, fb);
    case 8: return xlaunch(valu_stressor<8>, dim3(c.grid), dim3(threads), 0, s, e0, e1, c, out, iters, fa, fb);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_valu64_stressor(const KCtrl& c, double* out, uint32_t ilp, uint64_t iters64,
                                  double fa, uint32_t threads, hipStream_t s, hipEvent_t e0,
                                  hipEvent_t e1) {
  const uint32_t iters = (uint32_t)iters64;  // range checked by the caller
  switch (ilp) {
    case 1: return xlaunch(valu64_stressor<1>, dim3(c.grid), dim3(threads), 0, s, e0, e1, c, out, iters, fa);
    case 2: return xlaunch(valu64_stressor<2>, dim3(c.grid), dim3(threads), 0, s, e0, e1, c, out, iters, fa);
    case 4: return xlaunch(valu64_stressor<4>, dim3(c.grid), dim3(threads), 0, s, e0, e1, c, out, iters, fa);
    case 8: return xlaunch(valu64_stressor<8>, dim3(c.grid), dim3(threads), 0, s, e0, e1, c, out, iters, fa);
    default: return hipErrorInvalidValue;
  }
}

template <int DT>
static hipError_t launch_mfma_dt(const KCtrl& c, const void* a, const void* b, float* out,
                                 uint32_t accs, uint64_t iters, uint32_t threads, hipStream_t s,
                                 hipEvent_t e0, hipEvent_t e1) {
  switch (accs) {
    case 1: return xlaunch(mfma_stressor<DT, 1>, dim3(c.grid), dim3(threads), 0, s, e0, e1, c, a, b, out, iters);
    case 2: return xlaunch(mfma_stressor<DT, 2>, dim3(c.grid), dim3(threads), 0, s, e0, e1, c, a, b, out, iters);
    case 4: return xlaunch(mfma_stressor<DT, 4>, dim3(c.grid), dim3(threads), 0, s, e0, e1, c, a, b, out, iters);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_mfma_stressor(const KCtrl& c, int dtype, const void* a, const void* b, float* out,
                                uint32_t accs, uint64_t iters, uint32_t threads, hipStream_t s,
                                hipEvent_t e0, hipEvent_t e1) {
  switch (dtype) {
    case CI_DT_F32: return launch_mfma_dt<CI_DT_F32>(c, a, b, out, accs, iters, threads, s, e0, e1);
    case CI_DT_BF16: return launch_mfma_dt<CI_DT_BF16>(c, a, b, out, accs, iters, threads, s, e0, e1);
    case CI_DT_FP8E4M3: return launch_mfma_dt<CI_DT_FP8E4M3>(c, a, b, out, accs, iters, threads, s, e0, e1);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_chase_stressor(const KCtrl& c, const uint32_t* next, uint64_t n, uint32_t* end,
                                 uint32_t chains, uint64_t hops, uint32_t threads, hipStream_t s,
                                 hipEvent_t e0, hipEvent_t e1) {
  switch (chains) {
    case 1: return xlaunch(chase_stressor<1>, dim3(c.grid), dim3(threads), 0, s, e0, e1, c, next, n, end, hops);
    case 2: return xlaunch(chase_stressor<2>, dim3(c.grid), dim3(threads), 0, s, e0, e1, c, next, n, end, hops);
    case 4: return xlaunch(chase_stressor<4>, dim3(c.grid), dim3(threads), 0, s, e0, e1, c, next, n, end, hops);
    case 8: return xlaunch(chase_stressor<8>, dim3(c.grid), dim3(threads), 0, s, e0, e1, c, next, n, end, hops);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_dispatch_empty(uint32_t nwg, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  return xlaunch(empty_wg, dim3(nwg), dim3(64), 0, s, e0, e1);
}

hipError_t launch_dispatch_count(uint32_t nwg, uint64_t* counter, hipStream_t s, hipEvent_t e0,
                                 hipEvent_t e1) {
  return xlaunch(count_wg, dim3(nwg), dim3(64), 0, s, e0, e1, counter);
}

hipError_t launch_dispatch_announce(HostCtrl* host, hipStream_t s) {
  return xlaunch(announce_wg, dim3(1), dim3(64), 0, s, nullptr, nullptr, host);
}

hipError_t launch_hog(const KCtrl& c, uint32_t lds_bytes, uint32_t threads, hipStream_t s,
                      hipEvent_t e0, hipEvent_t e1) {
  return xlaunch(hog_kernel, dim3(c.grid), dim3(threads), lds_bytes, s, e0, e1, c, lds_bytes / 4u);
}

hipError_t launch_probe(uint32_t nwg, uint32_t* out, hipStream_t s) {
  return xlaunch(probe_kernel, dim3(nwg), dim3(64), 0, s, nullptr, nullptr, out);
}

hipError_t launch_mfma_probe(int dtype, const void* a, const void* b, const float* c, float* d,
                             uint32_t ntiles, hipStream_t s) {
  const uint8_t* pa = (const uint8_t*)a;
  const uint8_t* pb = (const uint8_t*)b;
  switch (dtype) {
    case CI_DT_F32: return xlaunch(mfma_probe_kernel<CI_DT_F32>, dim3(ntiles), dim3(64), 0, s, nullptr, nullptr, pa, pb, c, d);
    case CI_DT_BF16: return xlaunch(mfma_probe_kernel<CI_DT_BF16>, dim3(ntiles), dim3(64), 0, s, nullptr, nullptr, pa, pb, c, d);
    case CI_DT_FP8E4M3: return xlaunch(mfma_probe_kernel<CI_DT_FP8E4M3>, dim3(ntiles), dim3(64), 0, s, nullptr, nullptr, pa, pb, c, d);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ci
