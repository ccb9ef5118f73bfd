// Output checksums, per-tensor quantisation and the request-input fill used
// by the serving loop.
#include "internal.h"

namespace ci {
namespace {

// Checksums in two fixed-shape stages so the FP64 sum is the same on every
// run: stage 1 gives work-group p the contiguous range [p*len, (p+1)*len);
// each thread sums a fixed stride of it, then a fixed tree over the 256
// threads.  Stage 2 (one work-group) sums the partials the same way.
__device__ void block_reduce(uint64_t& bits, double& sum) {
  __shared__ uint64_t sb[256];
  __shared__ double ss[256];
  sb[threadIdx.x] = bits;
  ss[threadIdx.x] = sum;
  __syncthreads();
  for (uint32_t s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sb[threadIdx.x] += sb[threadIdx.x + s];
      ss[threadIdx.x] += ss[threadIdx.x + s];
    }
    __syncthreads();
  }
  bits = sb[0];
  sum = ss[0];
}

__global__ void __launch_bounds__(256) checksum_stage1(const float* __restrict__ x, uint64_t n,
                                                       uint64_t len, uint64_t* part_bits,
                                                       double* part_sum) {
  const uint64_t lo = (uint64_t)blockIdx.x * len;
  const uint64_t hi = lo + len < n ? lo + len : n;
  uint64_t bits = 0;
  double sum = 0.0;
  for (uint64_t i = lo + threadIdx.x; i < hi; i += 256) {
    const float v = x[i];
    bits += (uint64_t)__float_as_uint(v);
    sum += (double)v;
  }
  block_reduce(bits, sum);
  if (threadIdx.x == 0) {
    part_bits[blockIdx.x] = bits;
    part_sum[blockIdx.x] = sum;
  }
}

__global__ void __launch_bounds__(256) checksum_stage2(const uint64_t* part_bits,
                                                       const double* part_sum, uint32_t nparts,
                                                       uint64_t* out_bits, double* out_sum) {
  uint64_t bits = 0;
  double sum = 0.0;
  for (uint32_t i = threadIdx.x; i < nparts; i += 256) {
    bits += part_bits[i];
    sum += part_sum[i];
  }
  block_reduce(bits, sum);
  if (threadIdx.x == 0) {
    *out_bits = bits;
    *out_sum = sum;
  }
}

__global__ void __launch_bounds__(256) amax_stage1(const float* __restrict__ x, uint64_t n,
                                                   uint64_t len, float* part) {
  __shared__ float sm[256];
  const uint64_t lo = (uint64_t)blockIdx.x * len;
  const uint64_t hi = lo + len < n ? lo + len : n;
  float m = 0.0f;
  for (uint64_t i = lo + threadIdx.x; i < hi; i += 256) m = fmaxf(m, fabsf(x[i]));
  sm[threadIdx.x] = m;
  __syncthreads();
  for (uint32_t s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sm[threadIdx.x] = fmaxf(sm[threadIdx.x], sm[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

__global__ void __launch_bounds__(256) amax_stage2(const float* part, uint32_t nparts, float* out) {
  __shared__ float sm[256];
  float m = 0.0f;
  for (uint32_t i = threadIdx.x; i < nparts; i += 256) m = fmaxf(m, part[i]);
  sm[threadIdx.x] = m;
  __syncthreads();
  for (uint32_t s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sm[threadIdx.x] = fmaxf(sm[threadIdx.x], sm[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sm[0];
}

// FP32 -> BF16, round to nearest even by integer arithmetic on the bit
// pattern; NaN -> quiet NaN of the same sign.
__device__ __forceinline__ uint16_t to_bf16(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)(((u >> 16) & 0x8000u) | 0x7FC0u);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__global__ void __launch_bounds__(256) to_bf16_kernel(const float* __restrict__ x, uint64_t n,
                                                      uint16_t* __restrict__ out) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    out[i] = to_bf16(x[i]);
}

// FP32 -> OCP E4M3FN with round-to-nearest-even and saturation at +-448.
// Normal range (|y| >= 2^-6): keep 3 of the 23 mantissa bits, rounding on the
// 20 dropped bits; subnormal range: |y| * 2^9 rounded to an integer (exact
// scaling, v_rndne rounding), which also yields 2^-6 (code 8) on carry.
__device__ __forceinline__ uint8_t to_e4m3(float y) {
  const uint32_t u = __float_as_uint(y);
  const uint8_t sign = (uint8_t)((u >> 24) & 0x80u);
  const uint32_t a = u & 0x7FFFFFFFu;
  if (a > 0x7F800000u) return sign | 0x7Fu;          // NaN
  if (a >= 0x43E00000u) return sign | 0x7Eu;         // >= 448 (incl. inf): saturate
  const int e = (int)(a >> 23) - 127;
  if (e >= -6) {
    const uint32_t m = a & 0x7FFFFFu;
    uint32_t code = ((uint32_t)(e + 7) << 3) | (m >> 20);
    const uint32_t rem = m & 0xFFFFFu;
    if (rem > 0x80000u || (rem == 0x80000u && (code & 1u))) ++code;
    if (code > 0x7Eu) code = 0x7Eu;
    return sign | (uint8_t)code;
  }
  const float s = __uint_as_float(a) * 512.0f;       // exact
  const uint32_t q = (uint32_t)__builtin_rintf(s);  // nearest, ties to even
  return sign | (uint8_t)q;
}

__global__ void __launch_bounds__(256) to_fp8_kernel(const float* __restrict__ x, uint64_t n,
                                                     const float* __restrict__ amax,
                                                     uint8_t* __restrict__ out) {
  const float m = *amax;
  const float inv = (m > 0.0f && m <= 3.402823466e38f) ? __fdiv_rn(448.0f, m) : 1.0f;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    out[i] = to_e4m3(__fmul_rn(x[i], inv));  // a lone product: nothing to contract
}

__device__ __forceinline__ float uniform_from_word(uint64_t z) {
#pragma clang fp contract(off)
  const float k = (float)(uint32_t)(z >> 40);  // 24-bit integer: exact
  const float scaled = k * 0x1.0p-23f;          // exact
  return scaled - 1.0f;                         // exact
}

// Request inputs of the serving loop: SplitMix64 (Steele, Lea and Flood,
// OOPSLA 2014) in counter form, word i of stream `seed` = mix(seed + (i+1)G),
// mapped to a uniform value on [-1, 1) with 24 random bits.
__global__ void __launch_bounds__(256) fill_uniform_kernel(float* __restrict__ dst, uint64_t n,
                                                           uint64_t seed) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    uint64_t z = seed + (i + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    dst[i] = uniform_from_word(z);
  }
}

uint32_t grid_for(uint64_t n) {
  uint64_t g = (n + 255) / 256;
  if (g > 16384) g = 16384;
  if (g == 0) g = 1;
  return (uint32_t)g;
}

}  // namespace

hipError_t launch_checksum_f32(const float* x, uint64_t n, uint64_t* part_bits, double* part_sum,
                               uint32_t nparts, uint64_t* out_bits, double* out_sum,
                               hipStream_t s) {
  const uint64_t len = n ? (n + nparts - 1) / nparts : 1;
  hipError_t e = xlaunch(checksum_stage1, dim3(nparts), dim3(256), 0, s, nullptr, nullptr, x, n, len,
                         part_bits, part_sum);
  if (e != hipSuccess) return e;
  return xlaunch(checksum_stage2, dim3(1), dim3(256), 0, s, nullptr, nullptr, part_bits, part_sum, nparts,
                 out_bits, out_sum);
}

hipError_t launch_amax_f32(const float* x, uint64_t n, float* part, uint32_t nparts, float* out,
                           hipStream_t s) {
  const uint64_t len = n ? (n + nparts - 1) / nparts : 1;
  hipError_t e = xlaunch(amax_stage1, dim3(nparts), dim3(256), 0, s, nullptr, nullptr, x, n, len, part);
  if (e != hipSuccess) return e;
  return xlaunch(amax_stage2, dim3(1), dim3(256), 0, s, nullptr, nullptr, part, nparts, out);
}

hipError_t launch_to_bf16(const float* x, uint64_t n, uint16_t* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  return xlaunch(to_bf16_kernel, dim3(grid_for(n)), dim3(256), 0, s, nullptr, nullptr, x, n, out);
}

hipError_t launch_to_fp8(const float* x, uint64_t n, const float* amax, uint8_t* out,
                         hipStream_t s) {
  if (n == 0) return hipSuccess;
  return xlaunch(to_fp8_kernel, dim3(grid_for(n)), dim3(256), 0, s, nullptr, nullptr, x, n, amax, out);
}

hipError_t launch_fill_uniform(float* dst, uint64_t n, uint64_t seed, hipStream_t s) {
  if (n == 0) return hipSuccess;
  return xlaunch(fill_uniform_kernel, dim3(grid_for(n)), dim3(256), 0, s, nullptr, nullptr, dst, n, seed);
}

}  // namespace ci
