// Device fill of the SplitMix64 counter-form streams drawn in synth/__init__.py.
// Word i of stream `seed` is mix(seed + (i + 1) * GAMMA) (Steele, Lea and
// Flood, OOPSLA 2014).  Only the uniform, scaled-uniform and uint32 draws
// are offered here; they are integer work, exact conversions and (for the
// scaled draw) two individually rounded FP32 operations, so host and device
// agree bit for bit.  Draws only: no arithmetic of the measured method
// lives here.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ __forceinline__ uint64_t splitmix_word(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ float uniform_of(uint64_t w) {
#pragma clang fp contract(off)
  const float k = (float)(uint32_t)(w >> 40);  // 24-bit integer: exact
  const float scaled = k * 0x1.0p-23f;          // exact
  return scaled - 1.0f;                         // exact
}

__global__ void __launch_bounds__(256) fill_uniform_f32(float* __restrict__ dst, uint64_t n,
                                                        uint64_t seed, uint64_t start) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint64_t w = splitmix_word(seed, start + i);
    dst[i] = uniform_of(w);
  }
}

// u * scale + offset with two FP32 roundings (no fused multiply-add).
__device__ __forceinline__ float affine_of(float u, float scale, float offset) {
#pragma clang fp contract(off)
  const float t = u * scale;
  return t + offset;
}

__global__ void __launch_bounds__(256) fill_affine_f32(float* __restrict__ dst, uint64_t n,
                                                       uint64_t seed, uint64_t start, float scale,
                                                       float offset) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = affine_of(uniform_of(splitmix_word(seed, start + i)), scale, offset);
}

__global__ void __launch_bounds__(256) fill_u32(uint32_t* __restrict__ dst, uint64_t n,
                                                uint64_t seed, uint64_t start) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = (uint32_t)(splitmix_word(seed, start + i) >> 32);
}

unsigned grid_for(uint64_t n) {
  uint64_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  if (g == 0) g = 1;
  return (unsigned)g;
}

}  // namespace

extern "C" int synth_fill_uniform_f32(void* dst, uint64_t n, uint64_t seed, uint64_t start,
                                      void* stream) {
  if (n == 0) return 0;
  if (!dst) return (int)hipErrorInvalidValue;
  float* d = (float*)dst;
  void* argv[] = {&d, &n, &seed, &start};
  return (int)hipLaunchKernel((const void*)fill_uniform_f32, dim3(grid_for(n)), dim3(256), argv, 0,
                              (hipStream_t)stream);
}

extern "C" int synth_fill_u32(void* dst, uint64_t n, uint64_t seed, uint64_t start, void* stream) {
  if (n == 0) return 0;
  if (!dst) return (int)hipErrorInvalidValue;
  uint32_t* d = (uint32_t*)dst;
  void* argv[] = {&d, &n, &seed, &start};
  return (int)hipLaunchKernel((const void*)fill_u32, dim3(grid_for(n)), dim3(256), argv, 0,
                              (hipStream_t)stream);
}

extern "C" int synth_fill_affine_f32(void* dst, uint64_t n, uint64_t seed, uint64_t start, float scale,
                                     float offset, void* stream) {
  if (n == 0) return 0;
  if (!dst) return (int)hipErrorInvalidValue;
  float* d = (float*)dst;
  void* argv[] = {&d, &n, &seed, &start, &scale, &offset};
  return (int)hipLaunchKernel((const void*)fill_affine_f32, dim3(grid_for(n)), dim3(256), argv, 0,
                              (hipStream_t)stream);
}
