// Dense victims: GEMM C = s * A B^T on the matrix cores, and the BF16 GEMV
// y = W x.  The paper's shared-memory experiment uses a GEMM as the victim
// (Section 4.4.1, Figure 4) and its LLM decode victims are dominated by
// matrix-vector products that stream weights from memory (Sections 4.2-4.3).
//
// GEMM layout: A is M x K and B is N x K, both row-major (K contiguous), C is
// M x N FP32 row-major.  A 256-thread work-group owns a 128 x 128 tile of C;
// its four waves each own 64 x 64 (2 x 2 MFMA tiles of 32 x 32).  K is
// consumed in stages of 128 bytes per row, double-buffered in LDS through
// registers: the next stage's global loads are in flight while the current
// stage feeds the MFMAs.  Rows and K chunks past the matrix edges read as
// zero, so any M and N work; K * element size must be a multiple of 16.
#include "internal.h"

namespace ci {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

constexpr int kBM = 128, kBN = 128;
constexpr int kStageBytes = 128;                 // K bytes per stage per row
constexpr int kRowPitch = kStageBytes + 16;      // LDS row pitch (bank spread)
constexpr int kTileLds = 128 * kRowPitch;        // one operand, one stage

template <int DT>
struct Gemm;

template <>
struct Gemm<CI_DT_F32> {
  static constexpr int kElem = 4;
  static constexpr int kFragBytes = 4;     // per lane per MFMA operand
  static constexpr int kSub = kStageBytes / (2 * kFragBytes);
  __device__ static f32x16 mma(const uint8_t* pa, const uint8_t* pb, f32x16 acc) {
    const float a = *reinterpret_cast<const float*>(pa);
    const float b = *reinterpret_cast<const float*>(pb);
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
  }
};

template <>
struct Gemm<CI_DT_BF16> {
  static constexpr int kElem = 2;
  static constexpr int kFragBytes = 16;
  static constexpr int kSub = kStageBytes / (2 * kFragBytes);
  __device__ static f32x16 mma(const uint8_t* pa, const uint8_t* pb, f32x16 acc) {
    const bf16x8 a = *reinterpret_cast<const bf16x8*>(pa);
    const bf16x8 b = *reinterpret_cast<const bf16x8*>(pb);
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  }
};

template <>
struct Gemm<CI_DT_FP8E4M3> {
  static constexpr int kElem = 1;
  static constexpr int kFragBytes = 32;
  static constexpr int kSub = kStageBytes / (2 * kFragBytes);
  __device__ static f32x16 mma(const uint8_t* pa, const uint8_t* pb, f32x16 acc) {
    const i32x4 a0 = *reinterpret_cast<const i32x4*>(pa);
    const i32x4 a1 = *reinterpret_cast<const i32x4*>(pa + 16);
    const i32x4 b0 = *reinterpret_cast<const i32x4*>(pb);
    const i32x4 b1 = *reinterpret_cast<const i32x4*>(pb + 16);
    const i32x8 a = {a0[0], a0[1], a0[2], a0[3], a1[0], a1[1], a1[2], a1[3]};
    const i32x8 b = {b0[0], b0[1], b0[2], b0[3], b1[0], b1[1], b1[2], b1[3]};
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, acc, 0, 0, 0, 0, 0, 0);
  }
};

// Map the work-group index to a C tile so that the tiles one XCD works on
// are contiguous (work-groups are dealt to the 8 XCDs round-robin).
__device__ __forceinline__ void tile_of(uint32_t bid, uint32_t nbm, uint32_t nbn, uint32_t& tm,
                                        uint32_t& tn) {
  const uint32_t nb = nbm * nbn;
  uint32_t t = bid;
  if ((nb & 7u) == 0) t = (bid & 7u) * (nb >> 3) + (bid >> 3);
  tm = t / nbn;
  tn = t % nbn;
}

template <int DT>
__global__ void __launch_bounds__(256, 2) gemm_kernel(const uint8_t* __restrict__ A,
                                                      const uint8_t* __restrict__ B,
                                                      float* __restrict__ C, uint32_t M, uint32_t N,
                                                      uint32_t K, float scale) {
  using G = Gemm<DT>;
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  uint8_t* sA = smem;                  // [2][128][kRowPitch]
  uint8_t* sB = smem + 2 * kTileLds;   // [2][128][kRowPitch]
  const uint32_t nbm = (M + kBM - 1) / kBM, nbn = (N + kBN - 1) / kBN;
  uint32_t tm, tn;
  tile_of(blockIdx.x, nbm, nbn, tm, tn);
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wid = tid >> 6;
  const uint32_t wm = wid >> 1, wn = wid & 1u;   // wave's 64x64 sub-tile
  const uint64_t rowBytes = (uint64_t)K * G::kElem;
  const uint32_t nstages = (uint32_t)((rowBytes + kStageBytes - 1) / kStageBytes);

  // global -> register staging: thread loads 16 B at (row = tid/8 + 32 j, chunk = tid%8)
  const uint32_t lrow = tid >> 3, lchunk = tid & 7u;
  i32x4 ra[4], rb[4];
  auto gload = [&](uint32_t st) {
    const uint64_t kb = (uint64_t)st * kStageBytes + lchunk * 16u;
    const bool kin = kb + 16 <= rowBytes;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t r = lrow + 32u * j;
      const uint32_t gm = tm * kBM + r, gn = tn * kBN + r;
      ra[j] = (kin && gm < M) ? *reinterpret_cast<const i32x4*>(A + gm * rowBytes + kb) : i32x4{0, 0, 0, 0};
      rb[j] = (kin && gn < N) ? *reinterpret_cast<const i32x4*>(B + gn * rowBytes + kb) : i32x4{0, 0, 0, 0};
    }
  };
  auto sstore = [&](uint32_t buf) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t r = lrow + 32u * j;
      *reinterpret_cast<i32x4*>(sA + buf * kTileLds + r * kRowPitch + lchunk * 16u) = ra[j];
      *reinterpret_cast<i32x4*>(sB + buf * kTileLds + r * kRowPitch + lchunk * 16u) = rb[j];
    }
  };

  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;

  gload(0);
  sstore(0);
  __syncthreads();
  const uint32_t frow = lane & 31u, fk = (lane >> 5) * G::kFragBytes;
  for (uint32_t st = 0; st < nstages; ++st) {
    const uint32_t buf = st & 1u;
    if (st + 1 < nstages) gload(st + 1);
    const uint8_t* a0 = sA + buf * kTileLds + (wm * 64 + frow) * kRowPitch + fk;
    const uint8_t* b0 = sB + buf * kTileLds + (wn * 64 + frow) * kRowPitch + fk;
#pragma unroll
    for (int s = 0; s < G::kSub; ++s) {
      const uint32_t ko = s * 2 * G::kFragBytes;
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = G::mma(a0 + i * 32 * kRowPitch + ko, b0 + j * 32 * kRowPitch + ko, acc[i][j]);
    }
    if (st + 1 < nstages) sstore(buf ^ 1u);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const uint32_t col = tn * kBN + wn * 64 + j * 32 + (lane & 31u);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const uint32_t row = tm * kBM + wm * 64 + i * 32 + 8u * (v / 4) + 4u * (lane >> 5) + (v % 4);
        if (row < M && col < N) C[(uint64_t)row * N + col] = acc[i][j][v] * scale;
      }
    }
}

// Large-tile GEMM: one work-group per CU owns a 256 x 256 tile of C, with
// WAVES waves in a 2 x WAVES/2 grid: each wave owns 128 x (512/WAVES)
// (4 x 1024/(32 WAVES) MFMA tiles of 32 x 32), so every A fragment read from
// LDS feeds several MFMAs.  With 8 waves two share each SIMD, so one wave's
// LDS reads and barrier waits overlap the other's MFMAs.  Two 72 KiB
// K-stages of A and B are double-buffered in LDS (144 KiB of the CU's
// 160 KiB), filled through registers while the other stage computes.
constexpr int kBig = 256;
constexpr int kBigTileLds = kBig * kRowPitch;    // one operand, one stage
constexpr int kBigWaves = 8;

template <int DT, int WAVES>
__global__ void __launch_bounds__(64 * WAVES, 1) gemm256_kernel(const uint8_t* __restrict__ A,
                                                                const uint8_t* __restrict__ B,
                                                                float* __restrict__ C, uint32_t M,
                                                                uint32_t N, uint32_t K, float scale) {
  using G = Gemm<DT>;
  constexpr int NT = 64 * WAVES;          // threads
  constexpr int WN = WAVES / 2;           // waves along N
  constexpr int JN = kBig / WN / 32;      // 32-wide MFMA tiles per wave along N
  constexpr int LR = kBig / (NT / 8);     // rows each thread stages per operand
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  uint8_t* sA = smem;                     // [2][256][kRowPitch]
  uint8_t* sB = smem + 2 * kBigTileLds;   // [2][256][kRowPitch]
  const uint32_t nbm = (M + kBig - 1) / kBig, nbn = (N + kBig - 1) / kBig;
  uint32_t tm, tn;
  tile_of(blockIdx.x, nbm, nbn, tm, tn);
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wid = tid >> 6;
  const uint32_t wm = wid / WN, wn = wid % WN;   // wave's 128 x (256/WN) sub-tile
  const uint64_t rowBytes = (uint64_t)K * G::kElem;
  const uint32_t nstages = (uint32_t)((rowBytes + kStageBytes - 1) / kStageBytes);
  // global -> register staging: thread loads 16 B at (row = tid/8 + NT/8 j, chunk = tid%8)
  const uint32_t lrow = tid >> 3, lchunk = tid & 7u;
  i32x4 ra[LR], rb[LR];
  auto gload = [&](uint32_t st) {
    const uint64_t kb = (uint64_t)st * kStageBytes + lchunk * 16u;
    const bool kin = kb + 16 <= rowBytes;
#pragma unroll
    for (int j = 0; j < LR; ++j) {
      const uint32_t r = lrow + (NT / 8) * j;
      const uint32_t gm = tm * kBig + r, gn = tn * kBig + r;
      ra[j] = (kin && gm < M) ? *reinterpret_cast<const i32x4*>(A + gm * rowBytes + kb) : i32x4{0, 0, 0, 0};
      rb[j] = (kin && gn < N) ? *reinterpret_cast<const i32x4*>(B + gn * rowBytes + kb) : i32x4{0, 0, 0, 0};
    }
  };
  auto sstore = [&](uint32_t buf) {
#pragma unroll
    for (int j = 0; j < LR; ++j) {
      const uint32_t r = lrow + (NT / 8) * j;
      *reinterpret_cast<i32x4*>(sA + buf * kBigTileLds + r * kRowPitch + lchunk * 16u) = ra[j];
      *reinterpret_cast<i32x4*>(sB + buf * kBigTileLds + r * kRowPitch + lchunk * 16u) = rb[j];
    }
  };
  f32x16 acc[4][JN];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < JN; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;

  gload(0);
  sstore(0);
  __syncthreads();
  const uint32_t frow = lane & 31u, fk = (lane >> 5) * G::kFragBytes;
  for (uint32_t st = 0; st < nstages; ++st) {
    const uint32_t buf = st & 1u;
    if (st + 1 < nstages) gload(st + 1);
    const uint8_t* a0 = sA + buf * kBigTileLds + (wm * 128 + frow) * kRowPitch + fk;
    const uint8_t* b0 = sB + buf * kBigTileLds + (wn * (kBig / WN) + frow) * kRowPitch + fk;
#pragma unroll
    for (int s = 0; s < G::kSub; ++s) {
      const uint32_t ko = s * 2 * G::kFragBytes;
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < JN; ++j)
          acc[i][j] = G::mma(a0 + i * 32 * kRowPitch + ko, b0 + j * 32 * kRowPitch + ko, acc[i][j]);
    }
    if (st + 1 < nstages) sstore(buf ^ 1u);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < JN; ++j) {
      const uint32_t col = tn * kBig + wn * (kBig / WN) + j * 32 + (lane & 31u);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const uint32_t row = tm * kBig + wm * 128 + i * 32 + 8u * (v / 4) + 4u * (lane >> 5) + (v % 4);
        if (row < M && col < N) C[(uint64_t)row * N + col] = acc[i][j][v] * scale;
      }
    }
}

// GEMV: wave w handles rows w, w + W, ...; lane l reads 16-byte chunks
// l, l + 64, ... of the row (8 BF16 each), four chunks in flight, and keeps
// an FP32 running sum; the 64 partial sums are combined by a fixed butterfly.
__device__ __forceinline__ float bf16lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

__device__ __forceinline__ float dot8(uint4 w, uint4 x, float acc) {
  acc = __builtin_fmaf(bf16lo(w.x), bf16lo(x.x), acc);
  acc = __builtin_fmaf(bf16hi(w.x), bf16hi(x.x), acc);
  acc = __builtin_fmaf(bf16lo(w.y), bf16lo(x.y), acc);
  acc = __builtin_fmaf(bf16hi(w.y), bf16hi(x.y), acc);
  acc = __builtin_fmaf(bf16lo(w.z), bf16lo(x.z), acc);
  acc = __builtin_fmaf(bf16hi(w.z), bf16hi(x.z), acc);
  acc = __builtin_fmaf(bf16lo(w.w), bf16lo(x.w), acc);
  acc = __builtin_fmaf(bf16hi(w.w), bf16hi(x.w), acc);
  return acc;
}

__global__ void __launch_bounds__(256) gemv_bf16_kernel(const uint16_t* __restrict__ W,
                                                        const uint16_t* __restrict__ x,
                                                        float* __restrict__ y, uint64_t n,
                                                        uint64_t k) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t gw = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t nw = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  const uint64_t nch = k / 8;   // 16-byte chunks per row
  const uint4* x4 = reinterpret_cast<const uint4*>(x);
  for (uint64_t r = gw; r < n; r += nw) {
    const uint4* w4 = reinterpret_cast<const uint4*>(W + r * k);
    float acc = 0.0f;
    uint64_t c = lane;
    for (; c + 192 < nch; c += 256) {
      uint4 w[4], xv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) w[u] = w4[c + 64 * u];
#pragma unroll
      for (int u = 0; u < 4; ++u) xv[u] = x4[c + 64 * u];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = dot8(w[u], xv[u], acc);
    }
    for (; c < nch; c += 64) acc = dot8(w4[c], x4[c], acc);
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) y[r] = acc;
  }
}

}  // namespace

hipError_t launch_gemm(int dtype, const void* a, const void* b, float* c, uint64_t m, uint64_t n,
                       uint64_t k, float scale, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  // Large tiles once they fill the chip (>= one 256x256 tile per CU).
  const uint64_t nbig = ((m + kBig - 1) / kBig) * ((n + kBig - 1) / kBig);
  if (nbig >= 256) {
    const uint32_t shm = 4 * kBigTileLds;
    const uint8_t* A = (const uint8_t*)a;
    const uint8_t* B = (const uint8_t*)b;
    constexpr int W = kBigWaves;
    switch (dtype) {
      case CI_DT_F32:
        return xlaunch(gemm256_kernel<CI_DT_F32, W>, dim3((uint32_t)nbig), dim3(64 * W), shm, s, e0, e1, A,
                       B, c, (uint32_t)m, (uint32_t)n, (uint32_t)k, scale);
      case CI_DT_BF16:
        return xlaunch(gemm256_kernel<CI_DT_BF16, W>, dim3((uint32_t)nbig), dim3(64 * W), shm, s, e0, e1, A,
                       B, c, (uint32_t)m, (uint32_t)n, (uint32_t)k, scale);
      case CI_DT_FP8E4M3:
        return xlaunch(gemm256_kernel<CI_DT_FP8E4M3, W>, dim3((uint32_t)nbig), dim3(64 * W), shm, s, e0, e1,
                       A, B, c, (uint32_t)m, (uint32_t)n, (uint32_t)k, scale);
      default: return hipErrorInvalidValue;
    }
  }
  const uint64_t nb = ((m + kBM - 1) / kBM) * ((n + kBN - 1) / kBN);
  const uint32_t shm = 4 * kTileLds;
  const uint8_t* A = (const uint8_t*)a;
  const uint8_t* B = (const uint8_t*)b;
  switch (dtype) {
    case CI_DT_F32:
      return xlaunch(gemm_kernel<CI_DT_F32>, dim3((uint32_t)nb), dim3(256), shm, s, e0, e1, A, B, c,
                     (uint32_t)m, (uint32_t)n, (uint32_t)k, scale);
    case CI_DT_BF16:
      return xlaunch(gemm_kernel<CI_DT_BF16>, dim3((uint32_t)nb), dim3(256), shm, s, e0, e1, A, B, c,
                     (uint32_t)m, (uint32_t)n, (uint32_t)k, scale);
    case CI_DT_FP8E4M3:
      return xlaunch(gemm_kernel<CI_DT_FP8E4M3>, dim3((uint32_t)nb), dim3(256), shm, s, e0, e1, A, B,
                     c, (uint32_t)m, (uint32_t)n, (uint32_t)k, scale);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_gemv_bf16(const uint16_t* w, const uint16_t* x, float* y, uint64_t n, uint64_t k,
                            hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  uint64_t g = (n + 3) / 4;   // one wave per row, four waves per work-group
  if (g > 8192) g = 8192;
  if (g == 0) g = 1;
  return xlaunch(gemv_bf16_kernel, dim3((uint32_t)g), dim3(256), 0, s, e0, e1, w, x, y, n, k);
}

}  // namespace ci
