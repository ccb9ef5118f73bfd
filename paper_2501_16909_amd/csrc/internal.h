// Internal declarations shared by the libcoloc translation units: the
// device-side stressor protocol (stressor_dev.h) and the host launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

#include <tuple>
#include <utility>

#include "../../include/coloc.h"

#include "stressor_dev.h"

namespace ci {

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
// mix: CI_HBM_TRIAD / READ / COPY / WRITE (anything else: triad); chunk:
// 16-byte accesses per lane and stream in one wave-chunk (1, 2 or 4)
// strided: the read-only mix takes fixed per-wave strides instead of tickets
hipError_t launch_stream_stressor(const KCtrl& c, uint32_t mix, uint32_t chunk, const float* b,
                                  const float* cc, float* a, uint64_t n, uint32_t threads,
                                  bool streaming, bool strided, hipStream_t s, hipEvent_t e0,
                                  hipEvent_t e1);
// in_kernel: the passes loop inside one launch (each wave re-sweeps its own
// chunks) instead of one launch per pass
hipError_t launch_triad_victim(const float* b, const float* c, float* a, uint64_t n,
                               uint32_t passes, bool in_kernel, uint32_t grid, hipStream_t s,
                               hipEvent_t e0, hipEvent_t e1);
hipError_t launch_cache_stressor(const KCtrl& c, const uint32_t* region, uint64_t region_words,
                                 uint64_t slice_words, uint32_t batch, uint32_t threads,
                                 hipStream_t s,
    hipEvent_t e0, hipEvent_t e1);
hipError_t launch_lds_stressor(const KCtrl& c, const uint32_t* window, uint32_t vw, uint32_t stride,
                               bool load_only, uint32_t threads, hipStream_t s, hipEvent_t e0,
                               hipEvent_t e1);
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
hipError_t launch_mfma_probe(int dtype, const void* a, const void* b, const float* c, float* d,
                             uint32_t ntiles, hipStream_t s);
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
