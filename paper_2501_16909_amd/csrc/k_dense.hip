// Dense victims: GEMM C = s * A B^T on the matrix cores, and the BF16 GEMV
// y = W x.  The paper's shared-memory experiment uses a GEMM as the victim
// (Section 4.4.1, Figure 4) and its LLM decode victims are dominated by
// matrix-vector products that stream weights from memory (Sections 4.2-4.3).
//
// GEMM layout: A is M x K and B is N x K, both row-major (K contiguous), C is
// M x N FP32 row-major.  Three kernels, one summation order (each output is
// the MFMA chain over K in increasing order, so they agree bit for bit):
//   gemm256d_kernel  256 x 256 tiles, direct global -> LDS loads into a
//                    4-stage ring; shapes with >= 256 tiles and K * element
//                    size a multiple of 64 bytes;
//   gemm256_kernel   256 x 256 tiles staged through registers, other
//                    shapes with >= 256 tiles;
//   gemm_kernel      128 x 128 tiles for smaller shapes: a 256-thread
//                    work-group, four waves of 64 x 64 (2 x 2 MFMA tiles of
//                    32 x 32), K in stages of 128 bytes per row
//                    double-buffered in LDS through registers.
// Rows and K chunks past the matrix edges read as zero (register-staged
// kernels) or only feed outputs that are not stored (ring kernel), so any M
// and N work; K * element size must be a multiple of 16.
#include <type_traits>

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

// Map the work-group index to a C tile.  Work-groups are dealt to the 8
// XCDs round-robin, so first each XCD gets a contiguous range of tile
// numbers t; then t runs down bands of 4 tile rows (column by column within
// a band), so the tiles an XCD computes at one time form a 4 x 8 block that
// shares 4 A panels and 8 B panels in that XCD's L2 (a 2 x 16 row-major
// block would need 18).
template <uint32_t kBand = 4>
__device__ __forceinline__ void tile_of(uint32_t bid, uint32_t nbm, uint32_t nbn, uint32_t& tm,
                                        uint32_t& tn) {
  const uint32_t nb = nbm * nbn;
  uint32_t t = bid;
  if ((nb & 7u) == 0) t = (bid & 7u) * (nb >> 3) + (bid >> 3);
  const uint32_t band = kBand * nbn, group = t / band;
  const uint32_t first = group * kBand, rows = min(nbm - first, kBand), r = t - group * band;
  tm = first + r % rows;
  tn = r / rows;
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


// Large-tile GEMM with direct global -> LDS loads (16 bytes per lane,
// lane l of a wave instruction filling bytes 16 l of a 1 KiB block) into a
// 4-deep ring of K-stages of 64 bytes per row: two or three later stages
// are in flight while a stage computes, without staging registers.  Rows are
// stored unpadded; the 16-byte chunk c of row r sits at chunk
// c ^ ((r >> 2) & 3), so the 32 rows a fragment read touches fall on
// distinct banks.  Eight waves (2 x 4, each 128 x 64; two per SIMD) read
// fragments into registers and issue the MFMAs; with two MFMA k-steps per
// stage or more (FP32, BF16) the reads of the next k-step overlap the
// current one's MFMAs.  One bare barrier per stage: each wave first waits
// for its own loads of the stage (s_waitcnt on the vector-memory counter),
// so after the barrier the whole stage is in LDS; a fence there would also
// wait for the later stages' loads.  Needs K * element size to be a
// multiple of 64 bytes; the register-staged kernel above takes the rest.
// What bounds it: while MFMAs run, a SIMD takes in about one 1 KiB fragment
// load from LDS per 64 cycles, and a 128 x 64 wave tile issues six per eight
// 32 x 32 MFMAs, which caps the matrix core near two thirds of its rate even
// with no memory traffic or barriers (measured); larger wave tiles need more
// registers than two waves per SIMD have.
// Four slots of 32 KiB: 128 KiB of the CU's 160 KiB, leaving 32 KiB for a
// co-resident stressor work-group.  Five slots (loads three stages ahead)
// ran at the same rate within run-to-run spread, but fill the whole LDS, so
// no work-group holding any LDS could share a CU with the victim.
constexpr int kRingStages = 4;
constexpr int kDStage = 64;                         // K bytes per stage per row
constexpr int kDOperand = kBig * kDStage;           // one operand, one stage (16 KiB)
constexpr int kDSlot = 2 * kDOperand;               // A and B of one stage
static_assert(kRingStages * kDSlot <= 128 * 1024, "the ring must leave LDS for a co-resident work-group");

__device__ __forceinline__ uint32_t dswz(uint32_t row, uint32_t byte) {
  return row * kDStage + ((((byte >> 4) ^ (row >> 2)) & 3u) << 4) + (byte & 15u);
}

// One MFMA operand fragment per lane, read from a swizzled LDS stage.
template <int DT> struct Frag;
template <> struct Frag<CI_DT_F32> {
  using T = float;
  __device__ static T ld(const uint8_t* p, uint32_t row, uint32_t kb) {
    return *reinterpret_cast<const float*>(p + dswz(row, kb));
  }
  __device__ static f32x16 mma(T a, T b, f32x16 c) { return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0); }
};
template <> struct Frag<CI_DT_BF16> {
  using T = bf16x8;
  __device__ static T ld(const uint8_t* p, uint32_t row, uint32_t kb) {
    return *reinterpret_cast<const bf16x8*>(p + dswz(row, kb));
  }
  __device__ static f32x16 mma(T a, T b, f32x16 c) { return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0); }
};
template <> struct Frag<CI_DT_FP8E4M3> {
  using T = i32x8;
  __device__ static T ld(const uint8_t* p, uint32_t row, uint32_t kb) {
    const i32x4 a0 = *reinterpret_cast<const i32x4*>(p + dswz(row, kb));
    const i32x4 a1 = *reinterpret_cast<const i32x4*>(p + dswz(row, kb + 16));
    return i32x8{a0[0], a0[1], a0[2], a0[3], a1[0], a1[1], a1[2], a1[3]};
  }
  __device__ static f32x16 mma(T a, T b, f32x16 c) {
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 0, 0, 0);
  }
};

// BAND: tile rows per band of the tile order (tile_of).
template <int DT, uint32_t BAND>
__global__ void __launch_bounds__(512, 1) gemm256d_kernel(const uint8_t* __restrict__ A,
                                                          const uint8_t* __restrict__ B,
                                                          float* __restrict__ C, uint32_t M,
                                                          uint32_t N, uint32_t K, float scale) {
  using G = Gemm<DT>;
  constexpr int WN = 4, JN = 2;           // 8 waves: 2 x 4, each 128 x 64
  extern __shared__ __attribute__((aligned(1024))) uint8_t smem[];
  const uint32_t nbm = (M + kBig - 1) / kBig, nbn = (N + kBig - 1) / kBig;
  uint32_t tm, tn;
  tile_of<BAND>(blockIdx.x, nbm, nbn, tm, tn);
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wid = tid >> 6;
  const uint32_t wm = wid / WN, wn = wid % WN;
  const uint64_t rowBytes = (uint64_t)K * G::kElem;
  const uint32_t nstages = (uint32_t)(rowBytes / kDStage);
  // Wave w fills 1 KiB blocks w and w + 8 of each operand (16 blocks of 16
  // rows); lane l lands on row 16 q + l / 4, physical chunk l % 4.
  uint32_t lrow[2], lchunk[2];
  const uint8_t* srcA[2];
  const uint8_t* srcB[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const uint32_t q = wid + 8u * h;
    lrow[h] = 16u * q + (lane >> 2);
    lchunk[h] = ((lane & 3u) ^ (lrow[h] >> 2)) & 3u;    // logical chunk for this slot
    const uint32_t gm = min(tm * kBig + lrow[h], M - 1), gn = min(tn * kBig + lrow[h], N - 1);
    srcA[h] = A + (uint64_t)gm * rowBytes + lchunk[h] * 16u;
    srcB[h] = B + (uint64_t)gn * rowBytes + lchunk[h] * 16u;
  }
  auto issue = [&](uint32_t st) {
    uint8_t* slot = smem + (st % kRingStages) * kDSlot;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint32_t blk = (wid + 8u * h) * 1024u;
      __builtin_amdgcn_global_load_lds(srcA[h] + (uint64_t)st * kDStage, slot + blk, 16, 0, 0);
      __builtin_amdgcn_global_load_lds(srcB[h] + (uint64_t)st * kDStage, slot + kDOperand + blk, 16, 0, 0);
    }
  };
  f32x16 acc[4][JN];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < JN; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;
  const uint32_t frow = lane & 31u, fk = (lane >> 5) * G::kFragBytes;
  constexpr int NS = kDStage / (2 * G::kFragBytes);   // MFMA k-steps per stage
  using F = Frag<DT>;
  // Wait until this wave's loads of stage t are done (at most `ahead`
  // later stages of 4 instructions each may be pending), then a bare
  // barrier: every wave's part of stage t is in LDS.  A fence would also
  // wait for the later stages' loads.
  auto wait_stage = [&](uint32_t t, uint32_t ahead) {
    const uint32_t after = min(nstages - 1, t + ahead) - t;
    if (after >= 3) __builtin_amdgcn_s_waitcnt(0x0F7C);        // vmcnt(12)
    else if (after == 2) __builtin_amdgcn_s_waitcnt(0x0F78);   // vmcnt(8)
    else if (after == 1) __builtin_amdgcn_s_waitcnt(0x0F74);   // vmcnt(4)
    else __builtin_amdgcn_s_waitcnt(0x0F70);                   // vmcnt(0)
    __builtin_amdgcn_s_barrier();
  };
  if constexpr (NS % 2 == 0) {
    // Two fragment buffers of one k-step each: k-step g + 1 is read from LDS
    // while the MFMAs of k-step g run, across stage boundaries too.  The
    // reads of a stage's last k-step are waited for after the next stage's
    // barrier, so that barrier frees the slot of the stage before: stage
    // t + P is issued at the barrier of stage t into the slot of t - 2.
    constexpr uint32_t P = kRingStages - 2;
    for (uint32_t st = 0; st < P && st < nstages; ++st) issue(st);
    typename F::T fa[2][4], fb[2][JN];
    auto read_ks = [&](uint32_t t, int s, auto buf) {
      constexpr int b = decltype(buf)::value;
      const uint8_t* slot = smem + (t % kRingStages) * kDSlot;
      const uint32_t kb = fk + s * 2 * G::kFragBytes;
#pragma unroll
      for (int i = 0; i < 4; ++i) fa[b][i] = F::ld(slot, wm * 128 + i * 32 + frow, kb);
#pragma unroll
      for (int j = 0; j < JN; ++j) fb[b][j] = F::ld(slot + kDOperand, wn * 64 + j * 32 + frow, kb);
    };
    // MFMAs of one k-step: the first (first = true), the others (rest = true)
    auto mma_part = [&](auto buf, bool first, bool rest) {
      constexpr int b = decltype(buf)::value;
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < JN; ++j)
          if ((i == 0 && j == 0) ? first : rest) acc[i][j] = F::mma(fa[b][i], fb[b][j], acc[i][j]);
    };
    // FP32 (eight k-steps per stage): each k-step's block is its first MFMA,
    // then the next k-step's reads, then its other MFMAs, fenced in that
    // order, so that the reads have seven MFMAs to land; left to itself the
    // compiler issues them after the block and waits for them at once.
    // Measured 4 % faster for FP32, 1-2 % slower for BF16, which keeps the
    // compiler's order.  Results are bit-identical either way.
    constexpr bool kPinReads = DT == CI_DT_F32;
    auto fence = [] {
      if constexpr (kPinReads) __builtin_amdgcn_sched_barrier(0);
    };
    using B0 = std::integral_constant<int, 0>;
    using B1 = std::integral_constant<int, 1>;
    // stage t, its first k-step already in buffer 0; with `more`, the last
    // k-step's MFMAs overlap the next stage's barrier and first reads
    auto stage_body = [&](uint32_t t, bool more) {
#pragma unroll
      for (int s = 0; s < NS; s += 2) {
        if constexpr (kPinReads) {
          mma_part(B0{}, true, false);
          fence();
        }
        read_ks(t, s + 1, B1{});
        fence();
        mma_part(B0{}, !kPinReads, true);
        fence();
        if constexpr (kPinReads) {
          mma_part(B1{}, true, false);
          fence();
        }
        if (s + 2 < NS) {
          read_ks(t, s + 2, B0{});
        } else if (more) {
          wait_stage(t + 1, P - 1);
          if (t + 1 + P < nstages) issue(t + 1 + P);
          read_ks(t + 1, 0, B0{});
        }
        fence();
        mma_part(B1{}, !kPinReads, true);
        fence();
      }
    };
    wait_stage(0, P - 1);
    if (P < nstages) issue(P);
    read_ks(0, 0, B0{});
    // no branch around the reads in the steady state, so that each MFMA
    // block waits only for its own buffer's reads
    uint32_t st = 0;
    for (; st + 1 < nstages; ++st) stage_body(st, true);
    stage_body(st, false);
  } else {
    // One k-step per stage (FP8): a single buffer, read then multiplied;
    // the barrier of stage st frees the slot of st - 1.
    for (uint32_t st = 0; st < kRingStages - 1 && st < nstages; ++st) issue(st);
    for (uint32_t st = 0; st < nstages; ++st) {
      wait_stage(st, kRingStages - 2);
      if (st + kRingStages - 1 < nstages) issue(st + kRingStages - 1);
      const uint8_t* slot = smem + (st % kRingStages) * kDSlot;
      typename F::T fa[NS][4], fb[NS][JN];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const uint32_t kb = fk + s * 2 * G::kFragBytes;
#pragma unroll
        for (int i = 0; i < 4; ++i) fa[s][i] = F::ld(slot, wm * 128 + i * 32 + frow, kb);
#pragma unroll
        for (int j = 0; j < JN; ++j) fb[s][j] = F::ld(slot + kDOperand, wn * 64 + j * 32 + frow, kb);
      }
#pragma unroll
      for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < JN; ++j) acc[i][j] = F::mma(fa[s][i], fb[s][j], acc[i][j]);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < JN; ++j) {
      const uint32_t col = tn * kBig + wn * 64 + j * 32 + (lane & 31u);
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
  if (nbig >= 256 && (k * (dtype == CI_DT_F32 ? 4 : dtype == CI_DT_BF16 ? 2 : 1)) % kDStage == 0) {
    const uint32_t shm = kRingStages * kDSlot;
    const uint8_t* A = (const uint8_t*)a;
    const uint8_t* B = (const uint8_t*)b;
    // Tile order: bands of 8 tile rows when every tile runs at once (one
    // tile per CU), of 4 otherwise -- the faster of the two in each case
    // (BF16 4096^3: 1042-1048 against 847-989 TF; 8192^3: 1108-1130
    // against 1074-1079 TF).
    const bool one_wave = nbig <= 256;
#define CI_GEMM_RING(DT)                                                                                  \
  return one_wave ? xlaunch(gemm256d_kernel<DT, 8>, dim3((uint32_t)nbig), dim3(512), shm, s, e0, e1, A, B, c, \
                            (uint32_t)m, (uint32_t)n, (uint32_t)k, scale)                                 \
                  : xlaunch(gemm256d_kernel<DT, 4>, dim3((uint32_t)nbig), dim3(512), shm, s, e0, e1, A, B, c, \
                            (uint32_t)m, (uint32_t)n, (uint32_t)k, scale)
    switch (dtype) {
      case CI_DT_F32: CI_GEMM_RING(CI_DT_F32);
      case CI_DT_BF16: CI_GEMM_RING(CI_DT_BF16);
      case CI_DT_FP8E4M3: CI_GEMM_RING(CI_DT_FP8E4M3);
      default: return hipErrorInvalidValue;
    }
#undef CI_GEMM_RING
  }
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
