// Kernels of the synthetic decode step: the stand-in for the paper's LLM
// decode victims (Sections 4.2-4.4; per-kernel latencies of one step as in
// Fig. 5).  A Llama-style decoder layer with random weights, batch <= 8.
//
// Weight streaming dominates a decode step, so the GEMV is the kernel that
// matters, and the step is built around it: the small element-wise stages
// ride inside the GEMVs instead of paying a launch (and a pipeline drain)
// each.
//
//   gemv_fused_kernel   BF16 weight rows x NB vectors, FP32 accumulation.
//     input  BF16: the vectors as given;
//            NORM: FP32 vectors RMS-normalised with a BF16 gain and rounded
//                  to BF16 while they are staged (every work-group computes
//                  the norms itself, in the same order as rmsnorm_kernel);
//     output PLAIN: FP32 rows, plus an optional residual (may alias);
//            SILU:  rows j and j + rows/2 of one wave are gate and up, the
//                   epilogue writes BF16 SiLU(gate) * up;
//            ROPE:  rows i and i + head_dim/2 of a head share a wave, the
//                   epilogue applies the rotary embedding and writes the
//                   query (FP32) or appends key and value (BF16) to the cache.
//   attn_partial_kernel  grouped-query attention over 64-position chunks:
//                        per chunk max, exp-sum and unnormalised output.
//   attn_combine_kernel  merges the chunks of one head, BF16 out.
//   rmsnorm_kernel, rope_append_kernel, silu_mul_kernel: the same stages as
//     stand-alone kernels (the unfused composition the fused path must
//     reproduce bit for bit; they share the arithmetic helpers below).
#include "internal.h"

#include <math.h>

#include <algorithm>

namespace ci {
namespace {

__device__ __forceinline__ float bf_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf_hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

// FP32 -> BF16 bits, round to nearest even; NaN -> quiet NaN of the same sign.
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)(((u >> 16) & 0x8000u) | 0x7FC0u);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ uint32_t pack2(uint16_t lo, uint16_t hi) {
  return (uint32_t)lo | ((uint32_t)hi << 16);
}

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ float wave_max_f(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  return v;
}

__device__ __forceinline__ float dot8(uint4 w, uint4 x, float acc) {
  acc = __builtin_fmaf(bf_lo(w.x), bf_lo(x.x), acc);
  acc = __builtin_fmaf(bf_hi(w.x), bf_hi(x.x), acc);
  acc = __builtin_fmaf(bf_lo(w.y), bf_lo(x.y), acc);
  acc = __builtin_fmaf(bf_hi(w.y), bf_hi(x.y), acc);
  acc = __builtin_fmaf(bf_lo(w.z), bf_lo(x.z), acc);
  acc = __builtin_fmaf(bf_hi(w.z), bf_hi(x.z), acc);
  acc = __builtin_fmaf(bf_lo(w.w), bf_lo(x.w), acc);
  acc = __builtin_fmaf(bf_hi(w.w), bf_hi(x.w), acc);
  return acc;
}

// ---------------------------------------------- arithmetic shared by paths
// Sum of squares of x[0..n) by a 256-thread work-group: thread t takes the
// float4s t, t + 256, ..., then the waves' sums are added in a fixed order.
// Uniform control flow required (barriers).
__device__ float block_sumsq_256(const float* __restrict__ x, uint32_t n, float* s_part) {
  const float4* x4 = reinterpret_cast<const float4*>(x);
  float ss = 0.0f;
  for (uint32_t i = threadIdx.x; i < n / 4; i += 256) {
    const float4 v = x4[i];
    ss = fmaf(v.x, v.x, ss);
    ss = fmaf(v.y, v.y, ss);
    ss = fmaf(v.z, v.z, ss);
    ss = fmaf(v.w, v.w, ss);
  }
  ss = wave_sum_f(ss);
  if ((threadIdx.x & 63u) == 0) s_part[threadIdx.x >> 6] = ss;
  __syncthreads();
  const float tot = (s_part[0] + s_part[1]) + (s_part[2] + s_part[3]);
  __syncthreads();
  return tot;
}

__device__ __forceinline__ float rms_factor(float sumsq, uint32_t n, float eps) {
  return 1.0f / sqrtf(sumsq / (float)n + eps);
}

__device__ __forceinline__ uint16_t norm_bf16(float x, float r, float g) {
#pragma clang fp contract(off)
  return f32_to_bf16_rne((x * r) * g);
}

// Pair i of a head turns by pos * base^(-2i/d): angle, cosine and sine in
// FP64, rounded to FP32; the rotation in FP32 without contraction.
__device__ __forceinline__ void rope_cos_sin(uint32_t pos, uint32_t i, uint32_t d, float base, float* cs,
                                             float* sn) {
  const double ang = (double)pos * pow((double)base, -2.0 * (double)i / (double)d);
  *cs = (float)cos(ang);
  *sn = (float)sin(ang);
}

__device__ __forceinline__ void rope_apply(float x1, float x2, float cs, float sn, float* y1, float* y2) {
#pragma clang fp contract(off)
  *y1 = x1 * cs - x2 * sn;
  *y2 = x2 * cs + x1 * sn;
}

__device__ __forceinline__ float silu_mul_f(float g, float u) {
#pragma clang fp contract(off)
  return g / (1.0f + expf(-g)) * u;
}

// ---------------------------------------------------------------- RMSNorm
// One 256-thread work-group per row; n a multiple of 4.
__global__ void __launch_bounds__(256) rmsnorm_kernel(const float* __restrict__ x,
                                                      const uint16_t* __restrict__ g,
                                                      uint16_t* __restrict__ y, uint32_t n,
                                                      float eps) {
  __shared__ float s_part[4];
  const float* xr = x + (size_t)blockIdx.x * n;
  const float r = rms_factor(block_sumsq_256(xr, n, s_part), n, eps);
  const float4* x4 = reinterpret_cast<const float4*>(xr);
  const uint2* g2 = reinterpret_cast<const uint2*>(g);
  uint2* y2 = reinterpret_cast<uint2*>(y + (size_t)blockIdx.x * n);
  for (uint32_t i = threadIdx.x; i < n / 4; i += 256) {
    const float4 v = x4[i];
    const uint2 gw = g2[i];
    y2[i] = make_uint2(pack2(norm_bf16(v.x, r, bf_lo(gw.x)), norm_bf16(v.y, r, bf_hi(gw.x))),
                       pack2(norm_bf16(v.z, r, bf_lo(gw.y)), norm_bf16(v.w, r, bf_hi(gw.y))));
  }
}

// ------------------------------------------------------------------- GEMV
constexpr int IN_BF16 = 0, IN_NORM = 1;
constexpr int EPI_PLAIN = 0, EPI_SILU = 1, EPI_ROPE = 2;

// The rows one wave computes at a time (a "unit"): PLAIN R consecutive rows;
// SILU / ROPE one row pair (R = 2).  For ROPE the lane that writes vector b
// (lane b) also carries the pair's cosine and sine.
template <int R, int EPI>
struct Unit {
  uint32_t row[R];
  bool live[R];
  uint32_t jp;             // pair index (SILU / ROPE)
  const uint4* wr[R];
  float cs, sn;
};

template <int NB, int R, int EPI, bool kRope = true>
__device__ __forceinline__ void map_unit(const GemvArgs& a, uint32_t unit, uint32_t lane, Unit<R, EPI>& u) {
  if constexpr (EPI == EPI_PLAIN) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      u.row[r] = unit * R + r;
      u.live[r] = u.row[r] < a.rows;
    }
  } else {
    const uint32_t npairs = a.rows / 2;
    u.jp = unit;
    const bool ok = unit < npairs;
    if constexpr (EPI == EPI_SILU) {
      u.row[0] = unit;
      u.row[1] = unit + npairs;
    } else {
      const uint32_t half = a.d / 2, head = unit / half, i = unit - head * half;
      u.row[0] = head * a.d + i;
      u.row[1] = u.row[0] + half;
    }
    u.live[0] = u.live[1] = ok;
  }
#pragma unroll
  for (int r = 0; r < R; ++r)
    u.wr[r] = reinterpret_cast<const uint4*>(a.w + (size_t)(u.live[r] ? u.row[r] : 0) * a.k);
  u.cs = 1.0f;
  u.sn = 0.0f;
  if constexpr (EPI == EPI_ROPE && kRope) {
    const uint32_t half = a.d / 2, head = u.jp / half;
    if (u.live[0] && lane < a.batch && head < a.nq + a.nkv)
      rope_cos_sin((uint32_t)a.pos[lane], u.jp - head * half, a.d, a.base, &u.cs, &u.sn);
  }
}

// 16-byte chunks c = 256 j + lane + 64 v (v < 4) of round j of the unit's rows.
template <int R, int EPI>
__device__ __forceinline__ void load_round(const Unit<R, EPI>& u, uint32_t j, uint32_t lane, uint32_t kc,
                                           uint4 (&wv)[R][4]) {
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const uint32_t c = 256u * j + lane + 64u * v;
      wv[r][v] = (u.live[r] && c < kc) ? u.wr[r][c] : make_uint4(0, 0, 0, 0);
    }
}

template <int NB, int R, int EPI>
__device__ __forceinline__ void epilogue(const GemvArgs& a, const Unit<R, EPI>& u, uint32_t lane,
                                         float (&acc)[R][NB]) {
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[r][b] = wave_sum_f(acc[r][b]);
  if constexpr (EPI == EPI_PLAIN) {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int b = 0; b < NB; ++b)
        if (lane == (uint32_t)(r * NB + b) && u.live[r] && (uint32_t)b < a.batch) {
          const size_t o = (size_t)b * a.rows + u.row[r];
          a.out[o] = (a.res ? a.res[o] : 0.0f) + acc[r][b];
        }
  } else if constexpr (EPI == EPI_SILU) {
    const uint32_t f = a.rows / 2;
#pragma unroll
    for (int b = 0; b < NB; ++b)
      if (lane == (uint32_t)b && u.live[0] && (uint32_t)b < a.batch)
        a.h[(size_t)b * f + u.jp] = f32_to_bf16_rne(silu_mul_f(acc[0][b], acc[1][b]));
  } else {
    const uint32_t half = a.d / 2, head = u.jp / half, i = u.jp - head * half;
#pragma unroll
    for (int b = 0; b < NB; ++b)
      if (lane == (uint32_t)b && u.live[0] && (uint32_t)b < a.batch) {
        const uint32_t pp = (uint32_t)a.pos[b];
        const float x1 = acc[0][b], x2 = acc[1][b];
        if (head < a.nq) {
          float y1, y2;
          rope_apply(x1, x2, u.cs, u.sn, &y1, &y2);
          float* dst = a.q_out + ((size_t)b * a.nq + head) * a.d;
          dst[i] = y1;
          dst[i + half] = y2;
        } else if (head < a.nq + a.nkv) {
          float y1, y2;
          rope_apply(x1, x2, u.cs, u.sn, &y1, &y2);
          uint16_t* dst = a.kc + (((size_t)b * a.nkv + (head - a.nq)) * a.max_ctx + pp) * a.d;
          dst[i] = f32_to_bf16_rne(y1);
          dst[i + half] = f32_to_bf16_rne(y2);
        } else {
          uint16_t* dst = a.vc + (((size_t)b * a.nkv + (head - a.nq - a.nkv)) * a.max_ctx + pp) * a.d;
          dst[i] = f32_to_bf16_rne(x1);
          dst[i + half] = f32_to_bf16_rne(x2);
        }
      }
  }
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[r][b] = 0.0f;
}

// Stage chunks c0 .. c0 + nch - 1 of the NB vectors into LDS (BF16 input,
// or FP32 input normalised with factors s_r and gain g); zeros for b >= batch.
template <int NB, int IN>
__device__ __forceinline__ void stage_tile(const GemvArgs& a, uint32_t c0, uint32_t nch, uint32_t tc,
                                           const float* s_r, uint4* xs) {
  for (uint32_t i = threadIdx.x; i < NB * nch; i += 256) {
    const uint32_t b = i / nch, c = i - b * nch;
    uint4 val = make_uint4(0, 0, 0, 0);
    if (b < a.batch) {
      if constexpr (IN == IN_BF16) {
        val = reinterpret_cast<const uint4*>(a.v + (size_t)b * a.k)[c0 + c];
      } else {
        const float4* xp = reinterpret_cast<const float4*>(a.x + (size_t)b * a.k) + 2 * (c0 + c);
        const float4 x0 = xp[0], x1 = xp[1];
        const uint4 gg = reinterpret_cast<const uint4*>(a.g)[c0 + c];
        const float r = s_r[b];
        val.x = pack2(norm_bf16(x0.x, r, bf_lo(gg.x)), norm_bf16(x0.y, r, bf_hi(gg.x)));
        val.y = pack2(norm_bf16(x0.z, r, bf_lo(gg.y)), norm_bf16(x0.w, r, bf_hi(gg.y)));
        val.z = pack2(norm_bf16(x1.x, r, bf_lo(gg.z)), norm_bf16(x1.y, r, bf_hi(gg.z)));
        val.w = pack2(norm_bf16(x1.z, r, bf_lo(gg.w)), norm_bf16(x1.w, r, bf_hi(gg.w)));
      }
    }
    xs[b * tc + c] = val;
  }
}

// out = W x (rows of BF16 weights times NB vectors), FP32 accumulation.
// Work-group: 4 waves.  K is walked in rounds of 256 16-byte chunks (lane l
// takes chunks l, l+64, l+128, l+192 of a round: 1 KiB contiguous per row
// per wave); the vectors are staged in LDS in tiles of TK elements (32 KiB),
// once per work-group, read by all four waves.  TC is a multiple of 256, so
// a round never straddles two tiles.  Each lane's products are summed in
// increasing chunk order, then over the 64 lanes by a butterfly: the result
// does not depend on NB, R or the grid.
//   One tile (k <= TK): the grid is persistent; wave gw takes units gw,
//     gw + 4 gridDim.x, ...; the next step's weights (next round, or round 0
//     of the next unit) are loaded before the current step's products.
//   Several tiles: one unit per wave, tiles staged in turn.
template <int NB, int R, int IN, int EPI>
__global__ void __launch_bounds__(256) gemv_fused_kernel(GemvArgs a, uint32_t units) {
  constexpr uint32_t TK = 16384 / NB;
  constexpr uint32_t TC = TK / 8;
  __shared__ uint4 xs[NB * TC];
  __shared__ float s_part[4];
  __shared__ float s_r[NB];
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t gw = blockIdx.x * 4u + (threadIdx.x >> 6);
  const uint32_t nwaves = gridDim.x * 4u;
  const uint32_t kc = a.k / 8;
  const uint32_t nrounds = (kc + 255) / 256;
  float acc[R][NB];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[r][b] = 0.0f;
  Unit<R, EPI> cur;
  uint4 wcur[R][4], wnext[R][4];
  map_unit<NB, R, EPI>(a, gw, lane, cur);
  load_round(cur, 0, lane, kc, wcur);
  if constexpr (IN == IN_NORM) {
#pragma unroll 1
    for (uint32_t b = 0; b < (uint32_t)NB; ++b) {
      float tot = 0.0f;
      if (b < a.batch) tot = block_sumsq_256(a.x + (size_t)b * a.k, a.k, s_part);
      if (threadIdx.x == 0) s_r[b] = b < a.batch ? rms_factor(tot, a.k, a.eps) : 0.0f;
    }
  }
  if (kc <= TC) {
    __syncthreads();
    stage_tile<NB, IN>(a, 0, kc, TC, s_r, xs);
    __syncthreads();
    uint32_t unit = gw, j = 0;
    while (unit < units) {
      const bool wrap = j + 1 == nrounds;
      const uint32_t nunit = wrap ? unit + nwaves : unit;
      if (nunit < units) {
        if (wrap) {
          Unit<R, EPI> t;      // weights only: the rotary factors come with the unit itself
          map_unit<NB, R, EPI, false>(a, nunit, lane, t);
          load_round(t, 0, lane, kc, wnext);
        } else {
          load_round(cur, j + 1, lane, kc, wnext);
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const uint32_t c = 256u * j + lane + 64u * v;
        if (c >= kc) break;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const uint4 xv = xs[b * TC + c];
#pragma unroll
          for (int r = 0; r < R; ++r) acc[r][b] = dot8(wcur[r][v], xv, acc[r][b]);
        }
      }
      if (wrap) {
        epilogue<NB, R, EPI>(a, cur, lane, acc);
        map_unit<NB, R, EPI>(a, nunit, lane, cur);
      }
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int v = 0; v < 4; ++v) wcur[r][v] = wnext[r][v];
      unit = nunit;
      j = wrap ? 0 : j + 1;
    }
    return;
  }
  for (uint32_t j = 0; j < nrounds; ++j) {
    const uint32_t cr = 256u * j;          // first chunk of the round
    const uint32_t c0 = cr - cr % TC;      // first chunk of its tile
    if (cr == c0) {
      __syncthreads();
      stage_tile<NB, IN>(a, c0, min(TC, kc - c0), TC, s_r, xs);
      __syncthreads();
    }
    if (j + 1 < nrounds) load_round(cur, j + 1, lane, kc, wnext);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const uint32_t c = cr + lane + 64u * v;
      if (c >= kc) break;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const uint4 xv = xs[b * TC + (c - c0)];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r][b] = dot8(wcur[r][v], xv, acc[r][b]);
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int v = 0; v < 4; ++v) wcur[r][v] = wnext[r][v];
  }
  if (gw < units) epilogue<NB, R, EPI>(a, cur, lane, acc);
}

// ------------------------------------------------------------- RoPE + cache
// Stand-alone form.  grid (batch, n_q + 2 n_kv), block head_dim / 2.
// qkv: batch x (n_q + 2 n_kv) heads x head_dim FP32 (query heads, key heads,
// value heads).  Cache (one layer): batch x n_kv x max_ctx x head_dim BF16.
__global__ void __launch_bounds__(128) rope_append_kernel(const float* __restrict__ qkv,
                                                          const int32_t* __restrict__ pos,
                                                          float* __restrict__ q_out,
                                                          uint16_t* __restrict__ kc,
                                                          uint16_t* __restrict__ vc, uint32_t nq,
                                                          uint32_t nkv, uint32_t d,
                                                          uint32_t max_ctx, float base) {
  const uint32_t b = blockIdx.x, h = blockIdx.y, i = threadIdx.x, half = d / 2;
  const uint32_t p = (uint32_t)pos[b];
  const float* src = qkv + ((size_t)b * (nq + 2 * nkv) + h) * d;
  const float x1 = src[i], x2 = src[i + half];
  if (h >= nq + nkv) {
    uint16_t* dst = vc + (((size_t)b * nkv + (h - nq - nkv)) * max_ctx + p) * d;
    dst[i] = f32_to_bf16_rne(x1);
    dst[i + half] = f32_to_bf16_rne(x2);
    return;
  }
  float cs, sn, y1, y2;
  rope_cos_sin(p, i, d, base, &cs, &sn);
  rope_apply(x1, x2, cs, sn, &y1, &y2);
  if (h < nq) {
    float* dst = q_out + ((size_t)b * nq + h) * d;
    dst[i] = y1;
    dst[i + half] = y2;
  } else {
    uint16_t* dst = kc + (((size_t)b * nkv + (h - nq)) * max_ctx + p) * d;
    dst[i] = f32_to_bf16_rne(y1);
    dst[i + half] = f32_to_bf16_rne(y2);
  }
}

// -------------------------------------------------------------- attention
// grid (chunks, n_kv, batch), block group * 64 (group = n_q / n_kv <= 16):
// wave w handles query head kvh * group + w over positions t0 .. t0 + 63
// of key/value head kvh.  The chunk's keys and values are staged in LDS
// with 16-byte loads (rows padded to D/2 + 4 words); lane t scores position
// t0 + t.  Output per (batch, head, chunk): {max, exp-sum, D unnormalised
// outputs}; an empty chunk (t0 > pos) writes {-inf, 0, 0...}.
template <int D>
__global__ void __launch_bounds__(1024) attn_partial_kernel(const float* __restrict__ q,
                                                            const uint16_t* __restrict__ kc,
                                                            const uint16_t* __restrict__ vc,
                                                            const int32_t* __restrict__ pos,
                                                            float* __restrict__ part, uint32_t nq,
                                                            uint32_t nkv, uint32_t max_ctx,
                                                            uint32_t nchunks, float scale) {
  constexpr uint32_t kRow4 = D / 8;            // uint4 per cached row
  constexpr uint32_t kPitch4 = kRow4 + 1;      // padded, in uint4
  constexpr uint32_t kPitchW = 4 * kPitch4;    // in 32-bit words
  constexpr uint32_t kWPL = D / 128;           // value words per lane
  __shared__ uint4 ks[64 * kPitch4];
  __shared__ uint4 vs[64 * kPitch4];
  __shared__ float4 qs[16 * D / 4];
  __shared__ float ps[16 * 64];
  const uint32_t chunk = blockIdx.x, kvh = blockIdx.y, b = blockIdx.z;
  const uint32_t group = blockDim.x >> 6, lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  const uint32_t h = kvh * group + w;
  const int32_t T = pos[b] + 1;
  const uint32_t t0 = chunk * 64u;
  float* dst = part + (((size_t)b * nq + h) * nchunks + chunk) * (D + 2);
  if ((int32_t)t0 >= T) {
    if (lane == 0) {
      dst[0] = -INFINITY;
      dst[1] = 0.0f;
    }
    for (uint32_t j = lane; j < D; j += 64) dst[2 + j] = 0.0f;
    return;
  }
  // the query first (D/4 <= 64 float4: one per lane), so its load overlaps
  // the chunk's
  const float4* qh = reinterpret_cast<const float4*>(q + ((size_t)b * nq + h) * D);
  const float4 qv = lane < D / 4 ? qh[lane] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  const size_t base = (((size_t)b * nkv + kvh) * max_ctx + t0) * D;
  const uint4* k4 = reinterpret_cast<const uint4*>(kc + base);
  const uint4* v4 = reinterpret_cast<const uint4*>(vc + base);
  // rounds of four 16-byte loads per tensor per thread, all in flight
  // before any is stored
  constexpr uint32_t kTotal = 64 * kRow4;      // uint4 per tensor per chunk
  for (uint32_t i0 = threadIdx.x; i0 < kTotal; i0 += 4 * blockDim.x) {
    uint4 kk[4], vv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t i = i0 + u * blockDim.x;
      const bool ok = i < kTotal && (int32_t)(t0 + i / kRow4) < T;
      kk[u] = ok ? k4[i] : make_uint4(0, 0, 0, 0);
      vv[u] = ok ? v4[i] : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t i = i0 + u * blockDim.x;
      if (i < kTotal) {
        const uint32_t t = i / kRow4, c = i - t * kRow4;
        ks[t * kPitch4 + c] = kk[u];
        vs[t * kPitch4 + c] = vv[u];
      }
    }
  }
  if (lane < D / 4) qs[w * (D / 4) + lane] = qv;
  __syncthreads();
  float s = 0.0f;
  const uint4* kr = ks + lane * kPitch4;
  const float4* qw = qs + w * (D / 4);
#pragma unroll 4
  for (uint32_t c = 0; c < kRow4; ++c) {
    const uint4 kw = kr[c];
    const float4 qa = qw[2 * c], qb = qw[2 * c + 1];
    s = fmaf(qa.x, bf_lo(kw.x), s);
    s = fmaf(qa.y, bf_hi(kw.x), s);
    s = fmaf(qa.z, bf_lo(kw.y), s);
    s = fmaf(qa.w, bf_hi(kw.y), s);
    s = fmaf(qb.x, bf_lo(kw.z), s);
    s = fmaf(qb.y, bf_hi(kw.z), s);
    s = fmaf(qb.z, bf_lo(kw.w), s);
    s = fmaf(qb.w, bf_hi(kw.w), s);
  }
  const bool valid = (int32_t)(t0 + lane) < T;
  s = valid ? s * scale : -INFINITY;
  const float m = wave_max_f(s);        // finite: position t0 is valid
  const float p = valid ? expf(s - m) : 0.0f;
  const float l = wave_sum_f(p);
  ps[w * 64 + lane] = p;
  __syncthreads();
  float o[2 * kWPL];
#pragma unroll
  for (uint32_t j = 0; j < 2 * kWPL; ++j) o[j] = 0.0f;
  const uint32_t* vw32 = reinterpret_cast<const uint32_t*>(vs);
#pragma unroll 4
  for (uint32_t t = 0; t < 64; ++t) {
    const float pt = ps[w * 64 + t];
#pragma unroll
    for (uint32_t u = 0; u < kWPL; ++u) {
      const uint32_t vw = vw32[t * kPitchW + lane + 64 * u];
      o[2 * u] = fmaf(pt, bf_lo(vw), o[2 * u]);
      o[2 * u + 1] = fmaf(pt, bf_hi(vw), o[2 * u + 1]);
    }
  }
  if (lane == 0) {
    dst[0] = m;
    dst[1] = l;
  }
  float2* d2 = reinterpret_cast<float2*>(dst + 2);
#pragma unroll
  for (uint32_t u = 0; u < kWPL; ++u) d2[lane + 64 * u] = make_float2(o[2 * u], o[2 * u + 1]);
}

// grid (n_q, batch), block 256: merge the chunks of one head.  Thread t
// takes chunk maxima t, t+256, ... (block maximum M), then per tile of 256
// chunks the weights e_c = exp(m_c - M) go to LDS and thread t accumulates
// dimension pair t mod (D/2) over chunks t / (D/2), + 256/(D/2), ...; the
// partial sums of the chunk groups are added in a fixed order.
template <int D>
__global__ void __launch_bounds__(256) attn_combine_kernel(const float* __restrict__ part,
                                                           const int32_t* __restrict__ pos,
                                                           uint16_t* __restrict__ out, uint32_t nq,
                                                           uint32_t nchunks) {
  constexpr uint32_t kPairs = D / 2;            // dimension pairs
  constexpr uint32_t kGroups = 256 / kPairs;    // chunk groups (4 for D=128, 2 for D=256)
  __shared__ float s_e[256];
  __shared__ float s_red[4];
  __shared__ float2 s_o[kGroups][kPairs];
  const uint32_t h = blockIdx.x, b = blockIdx.y, t = threadIdx.x;
  const uint32_t nc = (uint32_t)pos[b] / 64u + 1u;
  const float* src = part + ((size_t)b * nq + h) * nchunks * (D + 2);
  float mx = -INFINITY;
  for (uint32_t c = t; c < nc; c += 256) mx = fmaxf(mx, src[(size_t)c * (D + 2)]);
  mx = wave_max_f(mx);
  if ((t & 63u) == 0) s_red[t >> 6] = mx;
  __syncthreads();
  const float M = fmaxf(fmaxf(s_red[0], s_red[1]), fmaxf(s_red[2], s_red[3]));
  __syncthreads();
  const uint32_t dp = t % kPairs, grp = t / kPairs;
  float lsum = 0.0f;
  float2 o = make_float2(0.0f, 0.0f);
  for (uint32_t c0 = 0; c0 < nc; c0 += 256) {
    const uint32_t n = min(256u, nc - c0);
    float e = 0.0f;
    if (t < n) {
      const float* pc = src + (size_t)(c0 + t) * (D + 2);
      e = expf(pc[0] - M);
      lsum = fmaf(pc[1], e, lsum);
    }
    s_e[t] = e;
    __syncthreads();
#pragma unroll 4
    for (uint32_t c = grp; c < n; c += kGroups) {
      const float ec = s_e[c];
      const float2 v = reinterpret_cast<const float2*>(src + (size_t)(c0 + c) * (D + 2) + 2)[dp];
      o.x = fmaf(v.x, ec, o.x);
      o.y = fmaf(v.y, ec, o.y);
    }
    __syncthreads();
  }
  lsum = wave_sum_f(lsum);
  if ((t & 63u) == 0) s_red[t >> 6] = lsum;
  s_o[grp][dp] = o;
  __syncthreads();
  const float L = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
  if (t < kPairs) {
    float2 acc = s_o[0][t];
#pragma unroll
    for (uint32_t g = 1; g < kGroups; ++g) {
      acc.x += s_o[g][t].x;
      acc.y += s_o[g][t].y;
    }
    uint32_t* dst = reinterpret_cast<uint32_t*>(out + ((size_t)b * nq + h) * D);
    dst[t] = pack2(f32_to_bf16_rne(acc.x / L), f32_to_bf16_rne(acc.y / L));
  }
}

// ------------------------------------------------------------------- SiLU
// Stand-alone form.  gu: batch x 2f FP32 (gate columns, then up columns);
// h: batch x f BF16.
__global__ void __launch_bounds__(256) silu_mul_kernel(const float* __restrict__ gu,
                                                       uint16_t* __restrict__ h, uint32_t f,
                                                       uint32_t batch) {
  const uint64_t n = (uint64_t)batch * f;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) {
    const uint64_t b = i / f, j = i - b * f;
    h[i] = f32_to_bf16_rne(silu_mul_f(gu[b * 2 * f + j], gu[b * 2 * f + f + j]));
  }
}

// Work-groups of `kernel` (256 threads) that fit on the device at once:
// the size of a persistent grid.
uint32_t resident_wgs(const void* kernel) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, 256, 0) != hipSuccess)
    return 256;
  return (uint32_t)std::max(1, cus * std::max(per, 1));
}

template <int NB, int R, int IN, int EPI>
uint32_t resident_of() {
  static const uint32_t n = resident_wgs(reinterpret_cast<const void*>(gemv_fused_kernel<NB, R, IN, EPI>));
  return n;
}

template <int NB, int R, int IN, int EPI>
hipError_t gemv_launch(const GemvArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const uint32_t units = EPI == EPI_PLAIN ? (a.rows + R - 1) / R : a.rows / 2;
  uint32_t grid = (units + 3) / 4;
  const uint32_t tc = 2048 / NB;
  if (a.k / 8 <= tc) grid = std::min(grid, resident_of<NB, R, IN, EPI>());
  if (grid == 0) grid = 1;
  return xlaunch(gemv_fused_kernel<NB, R, IN, EPI>, dim3(grid), dim3(256), 0, s, e0, e1, a, units);
}

template <int NB, int IN, int EPI>
hipError_t gemv_rows_r(const GemvArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  // plain rows: one row per wave while the resident grid still has a wave
  // for every row, two rows otherwise
  if constexpr (EPI == EPI_PLAIN) {
    if (a.rows <= 4 * resident_of<NB, 1, IN, EPI>()) return gemv_launch<NB, 1, IN, EPI>(a, s, e0, e1);
  }
  return gemv_launch<NB, 2, IN, EPI>(a, s, e0, e1);
}

template <int IN, int EPI>
hipError_t gemv_nb(const GemvArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (a.batch <= 1) return gemv_rows_r<1, IN, EPI>(a, s, e0, e1);
  if (a.batch <= 2) return gemv_rows_r<2, IN, EPI>(a, s, e0, e1);
  if (a.batch <= 4) return gemv_rows_r<4, IN, EPI>(a, s, e0, e1);
  return gemv_rows_r<8, IN, EPI>(a, s, e0, e1);
}

}  // namespace

hipError_t launch_gemv_fused(const GemvArgs& a, int input_norm, int epilogue, hipStream_t s, hipEvent_t e0,
                             hipEvent_t e1) {
  if (a.batch == 0 || a.batch > 8 || a.rows == 0 || a.k == 0 || a.k % 8) return hipErrorInvalidValue;
  if (input_norm) {
    switch (epilogue) {
      case EPI_PLAIN: return gemv_nb<IN_NORM, EPI_PLAIN>(a, s, e0, e1);
      case EPI_SILU: return gemv_nb<IN_NORM, EPI_SILU>(a, s, e0, e1);
      case EPI_ROPE: return gemv_nb<IN_NORM, EPI_ROPE>(a, s, e0, e1);
      default: return hipErrorInvalidValue;
    }
  }
  switch (epilogue) {
    case EPI_PLAIN: return gemv_nb<IN_BF16, EPI_PLAIN>(a, s, e0, e1);
    case EPI_SILU: return gemv_nb<IN_BF16, EPI_SILU>(a, s, e0, e1);
    case EPI_ROPE: return gemv_nb<IN_BF16, EPI_ROPE>(a, s, e0, e1);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_rmsnorm_bf16(const float* x, const uint16_t* g, uint16_t* y, uint32_t rows,
                               uint32_t n, float eps, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  return xlaunch(rmsnorm_kernel, dim3(rows), dim3(256), 0, s, e0, e1, x, g, y, n, eps);
}

hipError_t launch_rope_append(const float* qkv, const int32_t* pos, float* q_out, uint16_t* kc,
                              uint16_t* vc, uint32_t batch, uint32_t nq, uint32_t nkv, uint32_t d,
                              uint32_t max_ctx, float base, hipStream_t s, hipEvent_t e0,
                              hipEvent_t e1) {
  return xlaunch(rope_append_kernel, dim3(batch, nq + 2 * nkv), dim3(d / 2), 0, s, e0, e1, qkv, pos,
                 q_out, kc, vc, nq, nkv, d, max_ctx, base);
}

hipError_t launch_attn_partial(const float* q, const uint16_t* kc, const uint16_t* vc,
                               const int32_t* pos, float* part, uint32_t batch, uint32_t nq,
                               uint32_t nkv, uint32_t d, uint32_t max_ctx, uint32_t nchunks,
                               uint32_t used_chunks, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const dim3 grid(used_chunks, nkv, batch), block(64 * (nq / nkv));
  const float scale = (float)(1.0 / sqrt((double)d));
  if (d == 128)
    return xlaunch(attn_partial_kernel<128>, grid, block, 0, s, e0, e1, q, kc, vc, pos, part, nq, nkv,
                   max_ctx, nchunks, scale);
  if (d == 256)
    return xlaunch(attn_partial_kernel<256>, grid, block, 0, s, e0, e1, q, kc, vc, pos, part, nq, nkv,
                   max_ctx, nchunks, scale);
  return hipErrorInvalidValue;
}

hipError_t launch_attn_combine(const float* part, const int32_t* pos, uint16_t* out, uint32_t batch,
                               uint32_t nq, uint32_t d, uint32_t nchunks, hipStream_t s, hipEvent_t e0,
                               hipEvent_t e1) {
  if (d == 128)
    return xlaunch(attn_combine_kernel<128>, dim3(nq, batch), dim3(256), 0, s, e0, e1, part, pos, out, nq,
                   nchunks);
  if (d == 256)
    return xlaunch(attn_combine_kernel<256>, dim3(nq, batch), dim3(256), 0, s, e0, e1, part, pos, out, nq,
                   nchunks);
  return hipErrorInvalidValue;
}

hipError_t launch_silu_mul(const float* gu, uint16_t* h, uint32_t f, uint32_t batch, hipStream_t s,
                           hipEvent_t e0, hipEvent_t e1) {
  const uint64_t n = (uint64_t)batch * f;
  uint64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  if (g == 0) g = 1;
  return xlaunch(silu_mul_kernel, dim3((uint32_t)g), dim3(256), 0, s, e0, e1, gu, h, f, batch);
}

}  // namespace ci
