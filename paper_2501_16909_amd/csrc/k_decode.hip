// Kernels of the synthetic decode step: the stand-in for the paper's LLM
// decode victims (Sections 4.2-4.4; per-kernel latencies of one step as in
// Fig. 5).  A Llama-style decoder layer with random weights, batch <= 8:
//
//   rmsnorm_kernel       RMS normalisation with gain, BF16 out
//   gemv_rows_kernel     BF16 weight rows x NB BF16 vectors, FP32 out, with
//                        an optional FP32 residual added in the epilogue
//   rope_append_kernel   rotary embedding (rotate-half) of queries and keys;
//                        keys and values appended to the BF16 cache
//   attn_partial_kernel  grouped-query attention over 64-position chunks of
//                        the cache: per chunk max, exp-sum and unnormalised
//                        output (split over the context so that one
//                        sequence fills the chip)
//   attn_combine_kernel  merges the chunks, BF16 out
//   silu_mul_kernel      SiLU(gate) * up, BF16 out
//
// Weight streaming dominates a decode step, so the GEMV is the kernel that
// matters: one wave per R rows, 16-byte coalesced weight loads, the NB
// input vectors staged in LDS per K tile and shared by every wave of the
// work-group, FP32 accumulation and a butterfly reduction.
#include "internal.h"

#include <math.h>

namespace ci {
namespace {

__device__ __forceinline__ float bf_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf_hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// FP32 -> BF16 bits, round to nearest even; NaN -> quiet NaN of the same sign.
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)(((u >> 16) & 0x8000u) | 0x7FC0u);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
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

// ---------------------------------------------------------------- RMSNorm
// One work-group of 256 threads per row; n a multiple of 4.
__global__ void __launch_bounds__(256) rmsnorm_kernel(const float* __restrict__ x,
                                                      const uint16_t* __restrict__ g,
                                                      uint16_t* __restrict__ y, uint32_t n,
                                                      float eps) {
  __shared__ float part[4];
  const float4* xr = reinterpret_cast<const float4*>(x + (size_t)blockIdx.x * n);
  const uint2* gr = reinterpret_cast<const uint2*>(g);
  uint2* yr = reinterpret_cast<uint2*>(y + (size_t)blockIdx.x * n);
  const uint32_t n4 = n / 4;
  float ss = 0.0f;
  for (uint32_t i = threadIdx.x; i < n4; i += 256) {
    const float4 v = xr[i];
    ss = fmaf(v.x, v.x, ss);
    ss = fmaf(v.y, v.y, ss);
    ss = fmaf(v.z, v.z, ss);
    ss = fmaf(v.w, v.w, ss);
  }
  ss = wave_sum_f(ss);
  if ((threadIdx.x & 63u) == 0) part[threadIdx.x >> 6] = ss;
  __syncthreads();
  const float tot = (part[0] + part[1]) + (part[2] + part[3]);
  const float r = 1.0f / sqrtf(tot / (float)n + eps);
  for (uint32_t i = threadIdx.x; i < n4; i += 256) {
    const float4 v = xr[i];
    const uint2 gw = gr[i];
    const uint16_t a = f32_to_bf16_rne(v.x * r * bf_lo(gw.x));
    const uint16_t b = f32_to_bf16_rne(v.y * r * bf_hi(gw.x));
    const uint16_t c = f32_to_bf16_rne(v.z * r * bf_lo(gw.y));
    const uint16_t d = f32_to_bf16_rne(v.w * r * bf_hi(gw.y));
    yr[i] = make_uint2((uint32_t)a | ((uint32_t)b << 16), (uint32_t)c | ((uint32_t)d << 16));
  }
}

// ------------------------------------------------------------------- GEMV
// out[b][row] = res[b][row] (if res) + sum_j W[row][j] * v[b][j]
// W: rows x k BF16 row-major; v: NB x k BF16; res, out: NB x rows FP32 (they
// may alias: each element is read and then written by the same lane).
// Work-group: 4 waves, wave w owns rows (4 * blockIdx.x + w) * R .. + R - 1.
// K is walked in tiles of TK elements; each tile of the NB vectors is staged
// in LDS (32 KiB) and read by every wave.  Lane l covers 16-byte chunks
// l, l + 64, l + 128, l + 192 of each 256-chunk step, so a wave's loads of a
// row are 1 KiB contiguous.
template <int NB, int R>
__global__ void __launch_bounds__(256) gemv_rows_kernel(const uint16_t* __restrict__ W,
                                                        const uint16_t* __restrict__ v,
                                                        const float* res, float* out,
                                                        uint32_t rows, uint32_t k) {
  constexpr uint32_t TK = 16384 / NB;   // elements per vector per tile
  constexpr uint32_t TC = TK / 8;       // 16-byte chunks per vector per tile
  __shared__ uint4 xs[NB * TC];
  const uint32_t lane = threadIdx.x & 63u, wid = threadIdx.x >> 6;
  const uint32_t row0 = (blockIdx.x * 4u + wid) * R;
  bool live[R];
  const uint4* wr[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    live[r] = row0 + r < rows;
    wr[r] = reinterpret_cast<const uint4*>(W + (size_t)(live[r] ? row0 + r : 0) * k);
  }
  float acc[R][NB];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[r][b] = 0.0f;
  const uint32_t kc = k / 8;            // chunks per row
  for (uint32_t c0 = 0; c0 < kc; c0 += TC) {
    const uint32_t nch = min(TC, kc - c0);
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < NB * nch; i += 256) {
      const uint32_t b = i / nch, c = i - b * nch;
      xs[b * TC + c] = reinterpret_cast<const uint4*>(v + (size_t)b * k)[c0 + c];
    }
    __syncthreads();
    for (uint32_t c = lane; c < nch; c += 256) {
      uint4 w[R][4];
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int u = 0; u < 4; ++u)
          w[r][u] = (live[r] && c + 64u * u < nch) ? wr[r][c0 + c + 64u * u] : make_uint4(0, 0, 0, 0);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (c + 64u * u >= nch) break;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const uint4 xv = xs[b * TC + c + 64u * u];
#pragma unroll
          for (int r = 0; r < R; ++r) acc[r][b] = dot8(w[r][u], xv, acc[r][b]);
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[r][b] = wave_sum_f(acc[r][b]);
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int b = 0; b < NB; ++b)
      if (lane == (uint32_t)(r * NB + b) && live[r]) {
        const size_t o = (size_t)b * rows + row0 + r;
        out[o] = (res ? res[o] : 0.0f) + acc[r][b];
      }
}

// ------------------------------------------------------------- RoPE + cache
// grid (batch, n_q + 2 n_kv), block head_dim / 2.  qkv: batch x (n_q + 2 n_kv)
// heads x head_dim FP32 (query heads, key heads, value heads).  Pair i of a
// head is (i, i + head_dim/2), turned by pos * base^(-2i/head_dim); the angle
// and its cosine and sine are taken in FP64 and rounded to FP32.  Cache
// (this layer): batch x n_kv x max_ctx x head_dim BF16.
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
  const double ang = (double)p * pow((double)base, -2.0 * (double)i / (double)d);
  const float cs = (float)cos(ang), sn = (float)sin(ang);
  const float y1 = x1 * cs - x2 * sn;
  const float y2 = x2 * cs + x1 * sn;
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
// of key/value head kvh.  Keys and values of the chunk are staged in LDS
// with an odd row pitch (D/2 + 1 words), so lane-per-position score reads
// hit distinct banks.  Output per (batch, head, chunk): {max, exp-sum,
// D unnormalised outputs}; an empty chunk (t0 > pos) writes {-inf, 0, 0...}.
template <int D>
__global__ void __launch_bounds__(1024) attn_partial_kernel(const float* __restrict__ q,
                                                            const uint16_t* __restrict__ kc,
                                                            const uint16_t* __restrict__ vc,
                                                            const int32_t* __restrict__ pos,
                                                            float* __restrict__ part, uint32_t nq,
                                                            uint32_t nkv, uint32_t max_ctx,
                                                            uint32_t nchunks, float scale) {
  constexpr uint32_t kW = D / 2;        // 32-bit words per row
  constexpr uint32_t kPitch = kW + 1;
  constexpr uint32_t kWPL = D / 128;    // value words per lane
  __shared__ uint32_t ks[64 * kPitch];
  __shared__ uint32_t vs[64 * kPitch];
  __shared__ float qs[16 * D];
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
  const size_t base = (((size_t)b * nkv + kvh) * max_ctx + t0) * D;
  const uint32_t* k32 = reinterpret_cast<const uint32_t*>(kc + base);
  const uint32_t* v32 = reinterpret_cast<const uint32_t*>(vc + base);
  for (uint32_t i = threadIdx.x; i < 64 * kW; i += blockDim.x) {
    const uint32_t t = i / kW, c = i - t * kW;
    const bool ok = (int32_t)(t0 + t) < T;
    ks[t * kPitch + c] = ok ? k32[i] : 0u;
    vs[t * kPitch + c] = ok ? v32[i] : 0u;
  }
  const float* qh = q + ((size_t)b * nq + h) * D;
  for (uint32_t j = lane; j < D; j += 64) qs[w * D + j] = qh[j];
  __syncthreads();
  float s = 0.0f;
  const uint32_t* kr = ks + lane * kPitch;
  const float2* q2 = reinterpret_cast<const float2*>(qs + w * D);
#pragma unroll 8
  for (uint32_t c = 0; c < kW; ++c) {
    const uint32_t kw = kr[c];
    const float2 qq = q2[c];
    s = fmaf(qq.x, bf_lo(kw), s);
    s = fmaf(qq.y, bf_hi(kw), s);
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
  for (uint32_t t = 0; t < 64; ++t) {
    const float pt = ps[w * 64 + t];
    const uint32_t* vr = vs + t * kPitch;
#pragma unroll
    for (uint32_t u = 0; u < kWPL; ++u) {
      const uint32_t vw = vr[lane + 64 * u];
      o[2 * u] = fmaf(pt, bf_lo(vw), o[2 * u]);
      o[2 * u + 1] = fmaf(pt, bf_hi(vw), o[2 * u + 1]);
    }
  }
  if (lane == 0) {
    dst[0] = m;
    dst[1] = l;
  }
#pragma unroll
  for (uint32_t u = 0; u < kWPL; ++u) {
    const uint32_t j = 2 * (lane + 64 * u);
    dst[2 + j] = o[2 * u];
    dst[2 + j + 1] = o[2 * u + 1];
  }
}

// grid (n_q, batch), block 64: merge the chunks of one head.  out: batch x
// (n_q * D) BF16, head h at columns h * D.
template <int D>
__global__ void __launch_bounds__(64) attn_combine_kernel(const float* __restrict__ part,
                                                          const int32_t* __restrict__ pos,
                                                          uint16_t* __restrict__ out, uint32_t nq,
                                                          uint32_t nchunks) {
  constexpr uint32_t kWPL = D / 128;
  const uint32_t h = blockIdx.x, b = blockIdx.y, lane = threadIdx.x;
  const uint32_t nc = ((uint32_t)pos[b] + 64u) / 64u;
  const float* src = part + ((size_t)b * nq + h) * nchunks * (D + 2);
  float M = -INFINITY;
  for (uint32_t c = 0; c < nc; ++c) M = fmaxf(M, src[c * (D + 2)]);
  float L = 0.0f;
  float o[2 * kWPL];
#pragma unroll
  for (uint32_t j = 0; j < 2 * kWPL; ++j) o[j] = 0.0f;
  for (uint32_t c = 0; c < nc; ++c) {
    const float* pc = src + c * (D + 2);
    const float e = expf(pc[0] - M);
    L = fmaf(pc[1], e, L);
#pragma unroll
    for (uint32_t u = 0; u < kWPL; ++u) {
      const uint32_t j = 2 * (lane + 64 * u);
      o[2 * u] = fmaf(pc[2 + j], e, o[2 * u]);
      o[2 * u + 1] = fmaf(pc[3 + j], e, o[2 * u + 1]);
    }
  }
  uint32_t* dst = reinterpret_cast<uint32_t*>(out + ((size_t)b * nq + h) * D);
#pragma unroll
  for (uint32_t u = 0; u < kWPL; ++u) {
    const uint16_t lo = f32_to_bf16_rne(o[2 * u] / L);
    const uint16_t hi = f32_to_bf16_rne(o[2 * u + 1] / L);
    dst[lane + 64 * u] = (uint32_t)lo | ((uint32_t)hi << 16);
  }
}

// ------------------------------------------------------------------- SiLU
// gu: batch x 2f FP32 (gate columns, then up columns); h: batch x f BF16.
__global__ void __launch_bounds__(256) silu_mul_kernel(const float* __restrict__ gu,
                                                       uint16_t* __restrict__ h, uint32_t f,
                                                       uint32_t batch) {
  const uint64_t n = (uint64_t)batch * f;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) {
    const uint64_t b = i / f, j = i - b * f;
    const float g = gu[b * 2 * f + j], u = gu[b * 2 * f + f + j];
    h[i] = f32_to_bf16_rne(g / (1.0f + expf(-g)) * u);
  }
}

template <int NB>
hipError_t gemv_nb(const uint16_t* w, const uint16_t* v, const float* res, float* out, uint32_t rows,
                   uint32_t k, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  constexpr int R = NB <= 2 ? 2 : 4;
  const uint32_t grid = (rows + 4 * R - 1) / (4 * R);
  return xlaunch(gemv_rows_kernel<NB, R>, dim3(grid), dim3(256), 0, s, e0, e1, w, v, res, out, rows, k);
}

}  // namespace

hipError_t launch_rmsnorm_bf16(const float* x, const uint16_t* g, uint16_t* y, uint32_t rows,
                               uint32_t n, float eps, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  return xlaunch(rmsnorm_kernel, dim3(rows), dim3(256), 0, s, e0, e1, x, g, y, n, eps);
}

hipError_t launch_gemv_rows(const uint16_t* w, const uint16_t* v, const float* res, float* out,
                            uint32_t rows, uint32_t k, uint32_t batch, hipStream_t s, hipEvent_t e0,
                            hipEvent_t e1) {
  switch (batch) {
    case 1: return gemv_nb<1>(w, v, res, out, rows, k, s, e0, e1);
    case 2: return gemv_nb<2>(w, v, res, out, rows, k, s, e0, e1);
    case 3: return gemv_nb<3>(w, v, res, out, rows, k, s, e0, e1);
    case 4: return gemv_nb<4>(w, v, res, out, rows, k, s, e0, e1);
    case 5: return gemv_nb<5>(w, v, res, out, rows, k, s, e0, e1);
    case 6: return gemv_nb<6>(w, v, res, out, rows, k, s, e0, e1);
    case 7: return gemv_nb<7>(w, v, res, out, rows, k, s, e0, e1);
    case 8: return gemv_nb<8>(w, v, res, out, rows, k, s, e0, e1);
    default: return hipErrorInvalidValue;
  }
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
    return xlaunch(attn_combine_kernel<128>, dim3(nq, batch), dim3(64), 0, s, e0, e1, part, pos, out, nq,
                   nchunks);
  if (d == 256)
    return xlaunch(attn_combine_kernel<256>, dim3(nq, batch), dim3(64), 0, s, e0, e1, part, pos, out, nq,
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
