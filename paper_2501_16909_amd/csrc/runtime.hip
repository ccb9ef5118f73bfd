// Host runtime of libcoloc: context, CU masks, stressor launch / stop,
// victim runs, checksums, quantisation and the sensitivity engine.
#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"
#include "runtime.h"

using namespace ci;

// ------------------------------------------------------------------ errors
namespace {
thread_local std::string g_err;
}

ci_status_t ci::set_err(ci_status_t st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

extern "C" const char* ci_last_error(void) { return g_err.c_str(); }


// ----------------------------------------------------------------- context
namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

const char* kResName[CI_RES_COUNT] = {"hbm", "l2", "mall", "vl1d", "lds", "valu_f32",
                                      "mfma_f32", "mfma_bf16", "mfma_fp8", "ptrchase",
                                      "dispatch", "occupancy", "valu_f64"};

}  // namespace

int ci::cus_for(const ci_ctx* ctx, double intensity) {
  // whole steps of one CU per XCD, so every XCD keeps the same share
  const int per = ctx->info.num_cus / ctx->info.num_xcds;
  return ctx->info.num_xcds * (int)lround(per * intensity);
}

bool ci::mask_covers_all_xcds(const ci_ctx* ctx, const uint32_t mask[8]) {
  const int nx = ctx->info.num_xcds;
  for (int x = 0; x < nx; ++x) {
    bool any = false;
    for (int b = x; b < ctx->info.num_cus && !any; b += nx) any = (mask[b / 32] >> (b % 32)) & 1u;
    if (!any) return false;
  }
  return true;
}

static void forget_stream(ci_ctx* ctx, hipStream_t s) {
  auto& v = ctx->queue_checked;
  v.erase(std::remove_if(v.begin(), v.end(),
                         [s](const ci_ctx::QueuePair& p) { return p.victim == s || p.stressor == s; }),
          v.end());
}

static hipStream_t new_masked_stream(ci_ctx* ctx, const std::array<uint32_t, 8>& key) {
  hipStream_t s = nullptr;
  if (hipExtStreamCreateWithCUMask(&s, 8, key.data()) != hipSuccess) {
    (void)hipGetLastError();  // do not leave the failure for the next call to find
    return nullptr;
  }
  ++ctx->queue_gen;
  return s;
}

static void destroy_stream(ci_ctx* ctx, hipStream_t s) {
  (void)hipStreamSynchronize(s);
  (void)hipStreamDestroy(s);
  forget_stream(ctx, s);
  ++ctx->queue_gen;
}

static bool stream_in_use(const ci_ctx* ctx, hipStream_t s) {
  if (ctx->active && ctx->active->ms == s) return true;
  for (const hipStream_t* h : ctx->held)
    if (*h == s) return true;
  return false;
}

hipStream_t ci::masked_stream(ci_ctx* ctx, const uint32_t mask[8]) {
  std::array<uint32_t, 8> key{};
  for (int i = 0; i < 8; ++i) key[i] = mask[i];
  auto it = ctx->masked.find(key);
  if (it != ctx->masked.end()) {
    ctx->masked_used[key] = ++ctx->use_clock;
    return it->second;
  }
  // Each CU-masked stream owns a hardware queue: keep only a few, dropping
  // the least recently used one that nothing holds (not the running
  // stressor's, not a measurement's victim stream) before making another.
  // When every cached stream is in use the cache grows past the limit.
  if (ctx->masked.size() >= kMaxMaskedStreams) {
    auto lru = ctx->masked.end();
    uint64_t oldest = UINT64_MAX;
    for (auto jt = ctx->masked.begin(); jt != ctx->masked.end(); ++jt) {
      if (stream_in_use(ctx, jt->second)) continue;
      const uint64_t u = ctx->masked_used[jt->first];
      if (u < oldest) {
        oldest = u;
        lru = jt;
      }
    }
    if (lru != ctx->masked.end()) {
      destroy_stream(ctx, lru->second);
      ctx->masked_used.erase(lru->first);
      ctx->masked.erase(lru);
    }
  }
  hipStream_t s = new_masked_stream(ctx, key);
  if (s) {
    ctx->masked[key] = s;
    ctx->masked_used[key] = ++ctx->use_clock;
  }
  return s;
}

// A new hardware queue for `mask`: the replacement is created while the old
// queue still exists, so that it cannot be handed the same queue slot.
hipStream_t ci::replace_masked_stream(ci_ctx* ctx, const uint32_t mask[8]) {
  std::array<uint32_t, 8> key{};
  for (int i = 0; i < 8; ++i) key[i] = mask[i];
  hipStream_t s = new_masked_stream(ctx, key);
  if (!s) return nullptr;
  auto it = ctx->masked.find(key);
  if (it != ctx->masked.end()) destroy_stream(ctx, it->second);
  ctx->masked[key] = s;
  ctx->masked_used[key] = ++ctx->use_clock;
  return s;
}

void ci::mask_for(const ci_ctx* ctx, int k, int complement, uint32_t mask[8]) {
  // CU-mask bit b selects CU (b / XCDs) of XCD (b mod XCDs) (interleaved
  // across dies), so the first k bits give every XCD floor(k/8) or ceil(k/8).
  const int n = ctx->info.num_cus;
  for (int i = 0; i < 8; ++i) mask[i] = 0;
  for (int b = 0; b < n && b < 256; ++b) {
    const bool in = complement ? (b >= k) : (b < k);
    if (in) mask[b / 32] |= 1u << (b % 32);
  }
}

extern "C" ci_status_t ci_init(int device, ci_ctx_t** out) {
  if (!out) return set_err(CI_ERR_INVALID_ARG, "ci_init: out is NULL");
  *out = nullptr;
  int ndev = 0;
  HIPCHK(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev)
    return set_err(CI_ERR_INVALID_ARG, "ci_init: device %d not in [0, %d)", device, ndev);
  HIPCHK(hipSetDevice(device));
  ci_ctx* ctx = new (std::nothrow) ci_ctx();
  if (!ctx) return set_err(CI_ERR_OOM, "ci_init: host allocation");
  ctx->device = device;
  hipDeviceProp_t prop;
  hipError_t e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) {
    delete ctx;
    return set_err(CI_ERR_HIP, "hipGetDeviceProperties: %s", hipGetErrorString(e));
  }
  int wall_khz = 0;
  (void)hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, device);
  ci_device_info_t& in = ctx->info;
  memset(&in, 0, sizeof(in));
  in.device = device;
  in.num_cus = prop.multiProcessorCount;
  in.wave_size = prop.warpSize;
  in.clock_khz = prop.clockRate;
  in.wall_clock_khz = wall_khz > 0 ? wall_khz : 100000;
  in.lds_bytes_per_cu = prop.maxSharedMemoryPerMultiProcessor;
  in.l2_bytes_per_xcd = prop.l2CacheSize;
  in.hbm_bytes = prop.totalGlobalMem;
  snprintf(in.arch, sizeof(in.arch), "%s", prop.gcnArchName);
  in.num_xcds = 8;
  if (in.num_cus > 256 || in.num_cus <= 0) {
    delete ctx;
    return set_err(CI_ERR_UNSUPPORTED, "ci_init: %d CUs (CU masks cover 256)", in.num_cus);
  }

  // pinned control block and result slots (host-coherent)
  if (hipHostMalloc((void**)&ctx->host, sizeof(HostCtrl), hipHostMallocCoherent) != hipSuccess ||
      hipHostMalloc((void**)&ctx->hres, 64 * sizeof(uint64_t), hipHostMallocCoherent) != hipSuccess) {
    ci_shutdown(ctx);
    return set_err(CI_ERR_OOM, "ci_init: pinned host allocation");
  }
  memset((void*)ctx->host, 0, sizeof(HostCtrl));
  memset((void*)ctx->hres, 0, 64 * sizeof(uint64_t));
  ctx->nparts = 1024;
  if (hipMalloc((void**)&ctx->part_bits, ctx->nparts * sizeof(uint64_t)) != hipSuccess ||
      hipMalloc((void**)&ctx->part_sum, ctx->nparts * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&ctx->amax_part, ctx->nparts * sizeof(float)) != hipSuccess ||
      hipMalloc((void**)&ctx->amax_out, 256) != hipSuccess ||
      hipMalloc((void**)&ctx->probe_buf, 65536 * sizeof(uint32_t)) != hipSuccess) {
    ci_shutdown(ctx);
    return set_err(CI_ERR_OOM, "ci_init: device scratch");
  }
  for (auto& ev : ctx->ev) {
    if (hipEventCreate(&ev) != hipSuccess) {
      ci_shutdown(ctx);
      return set_err(CI_ERR_HIP, "ci_init: hipEventCreate");
    }
  }
  if (hipStreamCreateWithFlags(&ctx->vstream, hipStreamNonBlocking) != hipSuccess) {
    ci_shutdown(ctx);
    return set_err(CI_ERR_HIP, "ci_init: victim stream");
  }
  if (ci_status_t sst = static_scratch_init(device); sst != CI_OK) {
    ci_shutdown(ctx);
    return sst;
  }

  // Peaks.  Published MI355X figures where they exist; elsewhere bytes or
  // flops per clock per unit times units times the peak engine clock, or,
  // where no figure describes the unit, a measured ceiling (marked so).
  const double f = (double)in.clock_khz * 1e3;
  const double cus = in.num_cus;
  in.peak[CI_RES_HBM] = 8.0e12;                         // HBM3E, published
  in.peak[CI_RES_L2] = 8.0 * 16 * 128 * f;              // 16 channels x 128 B/clk per XCD
  // Infinity Cache: measured ceiling.  The best of 60 launch shapes and
  // traffic mixes of the streaming kernel over footprints of 64-192 MiB
  // (beyond the 32 MB of L2, inside the 256 MB cache) is 7.65 TB/s; streams
  // from all XCDs reach no more from the Infinity Cache than from HBM, so
  // the XCD-to-IOD fabric, not the cache, bounds streaming.  The CDNA3
  // figure of 17.2 TB/s is not reached by any shape.
  in.peak[CI_RES_MALL] = 7.65e12;
  in.peak[CI_RES_VL1D] = cus * 64.0 * f;                // 64 B/clk per CU
  // LDS: the load path, one 64-lane 16-byte load (1 KiB) per 4 clocks =
  // 256 B/clk per CU (CDNA4 doubled CDNA3's 128).  The load-only stressor
  // reaches 247 (96.5 %).  Stores are slower (76 B/clk per CU measured, no
  // published figure), so the copy form (one load and one store of each
  // vector) is bounded near 2 / (1/256 + 1/76) = 117 B/clk, 46 % of this peak.
  in.peak[CI_RES_LDS] = cus * 256.0 * f;
  in.peak[CI_RES_VALU_F32] = cus * 4 * 16 * 2.0 * f;    // unpacked FMA: 16 lanes/clk/SIMD
  in.peak[CI_RES_MFMA_F32] = 157.3e12;                  // published dense
  in.peak[CI_RES_MFMA_BF16] = 2.5166e15;                // published dense (2.5 PF)
  in.peak[CI_RES_MFMA_FP8] = 5.0332e15;                 // published dense (5.0 PF)
  in.peak[CI_RES_PTRCHASE] = 0.0;
  in.peak[CI_RES_DISPATCH] = 0.0;
  in.peak[CI_RES_OCCUPANCY] = 0.0;
  in.peak[CI_RES_VALU_F64] = cus * 4 * 16 * f;          // FP64 multiplies: 16 lanes/clk/SIMD
  *out = ctx;
  return CI_OK;
}

extern "C" ci_status_t ci_shutdown(ci_ctx_t* ctx) {
  if (!ctx) return CI_OK;
  if (ctx->active) return set_err(CI_ERR_BUSY, "ci_shutdown: a stressor is still running");
  (void)hipSetDevice(ctx->device);
  for (auto& kv : ctx->masked) (void)hipStreamDestroy(kv.second);
  ctx->masked.clear();
  ctx->masked_used.clear();
  ctx->queue_checked.clear();
  ctx->queue_qualified.clear();
  if (ctx->vstream) (void)hipStreamDestroy(ctx->vstream);
  for (auto& ev : ctx->ev)
    if (ev) (void)hipEventDestroy(ev);
  // after a failed drain a stressor kernel may still read the stop word:
  // that pinned block is left allocated
  if (ctx->host && !ctx->drain_failed) (void)hipHostFree((void*)ctx->host);
  if (ctx->hres) (void)hipHostFree((void*)ctx->hres);
  if (ctx->part_bits) (void)hipFree(ctx->part_bits);
  if (ctx->part_sum) (void)hipFree(ctx->part_sum);
  if (ctx->amax_part) (void)hipFree(ctx->amax_part);
  if (ctx->amax_out) (void)hipFree(ctx->amax_out);
  if (ctx->probe_buf) (void)hipFree(ctx->probe_buf);
  for (auto& kv : ctx->dec_graphs) (void)hipGraphExecDestroy(kv.second);
  ctx->dec_graphs.clear();
  for (auto& ev : ctx->dec_ev)
    if (ev) (void)hipEventDestroy(ev);
  if (ctx->dec_pos_host) (void)hipHostFree(ctx->dec_pos_host);
  if (ctx->dec_pos_dev) (void)hipFree(ctx->dec_pos_dev);
  delete ctx;
  return CI_OK;
}

extern "C" ci_status_t ci_device_info(ci_ctx_t* ctx, ci_device_info_t* out) {
  if (!ctx || !out) return set_err(CI_ERR_INVALID_ARG, "ci_device_info: NULL argument");
  *out = ctx->info;
  return CI_OK;
}

extern "C" ci_status_t ci_peak_for(ci_ctx_t* ctx, ci_resource_t r, double* peak) {
  if (!ctx || !peak || (int)r < 0 || r >= CI_RES_COUNT)
    return set_err(CI_ERR_INVALID_ARG, "ci_peak_for: bad argument");
  *peak = ctx->info.peak[r];
  return CI_OK;
}

extern "C" ci_status_t ci_cu_mask(ci_ctx_t* ctx, float intensity, int complement, uint32_t mask[8],
                                  int* ncu) {
  if (!ctx || !mask) return set_err(CI_ERR_INVALID_ARG, "ci_cu_mask: NULL argument");
  if (!(intensity >= 0.0f && intensity <= 1.0f))
    return set_err(CI_ERR_INVALID_ARG, "ci_cu_mask: intensity %g not in [0, 1]", intensity);
  const int k = cus_for(ctx, intensity);
  mask_for(ctx, k, complement, mask);
  if (ncu) *ncu = complement ? ctx->info.num_cus - k : k;
  return CI_OK;
}

extern "C" ci_status_t ci_probe_placement(ci_ctx_t* ctx, const uint32_t* mask, uint32_t nwg,
                                          uint32_t* out_loc) {
  if (!ctx || !out_loc || nwg == 0) return set_err(CI_ERR_INVALID_ARG, "ci_probe_placement: bad argument");
  uint32_t full[8];
  if (!mask) {
    mask_for(ctx, ctx->info.num_cus, 0, full);
    mask = full;
  }
  if (!mask_covers_all_xcds(ctx, mask))
    return set_err(CI_ERR_INVALID_ARG, "ci_probe_placement: mask leaves an XCD without CUs");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t s = masked_stream(ctx, mask);
  if (!s) return set_err(CI_ERR_HIP, "hipExtStreamCreateWithCUMask failed");
  HIPCHK(launch_probe(nwg, out_loc, s));
  HIPCHK(hipStreamSynchronize(s));
  return CI_OK;
}

// ---------------------------------------------------------------- stressors
namespace {

struct Defaults {
  uint32_t threads, wg_per_cu, knob, vec;
  uint64_t iters;
  uint32_t chunk;
};

Defaults defaults_for(ci_resource_t r) {
  // Chosen from standalone sweeps on MI355X (work-groups per CU x threads):
  // the smallest occupancy within a few percent of the best rate, so that a
  // colocated victim can still be dispatched beside the stressor.
  switch (r) {
    // streaming stressors: 8 waves per CU, 4 x 16 bytes per lane and stream
    // in flight (the best HBM triad rate of 21 shapes, 81 % of the peak)
    case CI_RES_HBM: return {512, 1, CI_HBM_TRIAD, 0, 0, 4};
    case CI_RES_L2: return {512, 3, 0, 0, 0};
    case CI_RES_MALL: return {512, 1, CI_HBM_READ, 1, 0, 4};
    case CI_RES_VL1D: return {256, 4, 0, 0, 0};
    case CI_RES_LDS: return {1024, 1, 1, 4, 0};
    case CI_RES_VALU_F32: return {256, 4, 8, 0, 4096};
    case CI_RES_MFMA_F32:
    case CI_RES_MFMA_BF16:
    case CI_RES_MFMA_FP8: return {256, 2, 4, 0, 1024};
    case CI_RES_PTRCHASE: return {256, 1, 4, 0, 1024};
    case CI_RES_DISPATCH: return {64, 0, 0, 0, 1000000};
    case CI_RES_OCCUPANCY: return {256, 1, 64, 0, 0};
    case CI_RES_VALU_F64: return {256, 4, 4, 0, 4096};
    default: return {256, 1, 0, 0, 0};
  }
}

void resolve(ci_resource_t r, const ci_stressor_opts_t* in, ci_stressor_opts_t* o) {
  if (in) *o = *in;
  else memset(o, 0, sizeof(*o));
  const Defaults d = defaults_for(r);
  if (!o->threads) o->threads = d.threads;
  if (!o->wg_per_cu) o->wg_per_cu = d.wg_per_cu;
  if (!o->knob) o->knob = d.knob;
  if (!o->vec) o->vec = d.vec;
  if (!o->iters) o->iters = d.iters;
  if (!o->deadline_ms) o->deadline_ms = 2000;
  if (!o->chunk) o->chunk = d.chunk ? d.chunk : 2;
}

// Bytes moved per element by each HBM traffic mix (4-byte words).
double hbm_bytes_per_element(uint32_t mix) {
  switch (mix) {
    case CI_HBM_READ:
    case CI_HBM_COPY: return 8.0;
    case CI_HBM_WRITE: return 4.0;
    default: return 12.0;
  }
}

int mfma_dtype(ci_resource_t r) {
  return r == CI_RES_MFMA_F32 ? CI_DT_F32 : r == CI_RES_MFMA_BF16 ? CI_DT_BF16 : CI_DT_FP8E4M3;
}

int mfma_k(int dt) { return dt == CI_DT_F32 ? 2 : dt == CI_DT_BF16 ? 16 : 64; }

// Words one work-group reads per pass for the cache stressors (L2, vL1D):
// every work-group reads the whole region.
uint64_t cache_span_words(const ci_stressor_opts_t& o) { return o.n; }

ci_status_t check_opts(ci_ctx* ctx, ci_resource_t r, const ci_stressor_opts_t& o, uint32_t grid) {
  if (o.duty > 100) return set_err(CI_ERR_INVALID_ARG, "%s: duty %u%% > 100", kResName[r], o.duty);
  if (o.threads == 0 || o.threads > 1024 || o.threads % 64)
    return set_err(CI_ERR_INVALID_ARG, "%s: threads %u must be a multiple of 64 in [64, 1024]",
                   kResName[r], o.threads);
  if (r != CI_RES_LDS && o.access != 0)
    return set_err(CI_ERR_INVALID_ARG, "%s: access %u is an LDS option (must be 0)", kResName[r], o.access);
  switch (r) {
    case CI_RES_HBM:
    case CI_RES_MALL: {
      if (o.knob < CI_HBM_TRIAD || o.knob > CI_HBM_WRITE)
        return set_err(CI_ERR_INVALID_ARG, "%s: traffic mix %u is not one of CI_HBM_*", kResName[r], o.knob);
      if (o.chunk != 1 && o.chunk != 2 && o.chunk != 4)
        return set_err(CI_ERR_INVALID_ARG, "%s: chunk must be 1, 2 or 4", kResName[r]);
      // arrays each mix touches: triad b, c, a; read b, c; copy b, a; write a
      const bool need_b = o.knob != CI_HBM_WRITE;
      const bool need_c = o.knob == CI_HBM_TRIAD || o.knob == CI_HBM_READ;
      const bool need_a = o.knob != CI_HBM_READ;
      static const char* const kNeed[] = {"", "b, c and a", "b and c", "b and a", "a"};
      if ((need_b && !o.src0) || (need_c && !o.src1) || (need_a && !o.dst))
        return set_err(CI_ERR_INVALID_ARG, "%s: %s required", kResName[r], kNeed[o.knob]);
      if (o.n == 0) return set_err(CI_ERR_INVALID_ARG, "%s: n must be > 0", kResName[r]);
      if (((need_b ? (uintptr_t)o.src0 : 0) | (need_c ? (uintptr_t)o.src1 : 0) |
           (need_a ? (uintptr_t)o.dst : 0)) & 15)
        return set_err(CI_ERR_INVALID_ARG, "%s: arrays must be 16-byte aligned", kResName[r]);
      if (o.knob == CI_HBM_WRITE && o.n > (1ull << 32))
        return set_err(CI_ERR_INVALID_ARG, "%s: the write pattern is defined for n <= 2^32", kResName[r]);
      break;
    }
    case CI_RES_L2:
    case CI_RES_VL1D: {
      if (!o.src0) return set_err(CI_ERR_INVALID_ARG, "%s: region is required", kResName[r]);
      if ((uintptr_t)o.src0 & 15) return set_err(CI_ERR_INVALID_ARG, "%s: region must be 16-byte aligned", kResName[r]);
      const uint64_t span = cache_span_words(o);
      if (span / (4ull * o.threads) > 0xFFFFFFFFull)
        return set_err(CI_ERR_INVALID_ARG, "%s: region too large", kResName[r]);
      if (span == 0 || span % (4ull * o.threads))
        return set_err(CI_ERR_INVALID_ARG,
                       "%s: region of %llu words gives a per-work-group span of %llu words, which "
                       "must be a positive multiple of %u",
                       kResName[r], (unsigned long long)o.n, (unsigned long long)span, 4 * o.threads);
      break;
    }
    case CI_RES_LDS:
      if (!o.src0) return set_err(CI_ERR_INVALID_ARG, "lds: window (8192 words) is required");
      if (o.vec != 1 && o.vec != 2 && o.vec != 4) return set_err(CI_ERR_INVALID_ARG, "lds: vec must be 1, 2 or 4");
      if (o.knob == 0) return set_err(CI_ERR_INVALID_ARG, "lds: stride must be >= 1");
      if (o.access != CI_LDS_COPY && o.access != CI_LDS_LOAD)
        return set_err(CI_ERR_INVALID_ARG, "lds: access must be CI_LDS_COPY or CI_LDS_LOAD");
      if ((uint64_t)o.wg_per_cu * 65536 > ctx->info.lds_bytes_per_cu)
        return set_err(CI_ERR_INVALID_ARG, "lds: %u work-groups x 64 KiB exceed the CU's LDS", o.wg_per_cu);
      break;
    case CI_RES_VALU_F32:
      if (!o.dst) return set_err(CI_ERR_INVALID_ARG, "valu: dst is required");
      if (o.iters == 0 || o.iters > 0xFFFFFFFFull) return set_err(CI_ERR_INVALID_ARG, "valu: iters must be in [1, 2^32)");
      if (o.knob != 1 && o.knob != 2 && o.knob != 4 && o.knob != 8)
        return set_err(CI_ERR_INVALID_ARG, "valu: ILP must be 1, 2, 4 or 8");
      break;
    case CI_RES_VALU_F64:
      if (!o.dst) return set_err(CI_ERR_INVALID_ARG, "valu_f64: dst is required");
      if (o.knob != 1 && o.knob != 2 && o.knob != 4 && o.knob != 8)
        return set_err(CI_ERR_INVALID_ARG, "valu_f64: ILP must be 1, 2, 4 or 8");
      if (o.iters == 0 || o.iters > 0xFFFFFFFFull) return set_err(CI_ERR_INVALID_ARG, "valu_f64: iters must be in [1, 2^32)");
      break;
    case CI_RES_MFMA_F32:
    case CI_RES_MFMA_BF16:
    case CI_RES_MFMA_FP8:
      if (!o.src0 || !o.src1 || !o.dst) return set_err(CI_ERR_INVALID_ARG, "mfma: A, B and dst are required");
      if (o.knob != 1 && o.knob != 2 && o.knob != 4)
        return set_err(CI_ERR_INVALID_ARG, "mfma: accumulators must be 1, 2 or 4");
      break;
    case CI_RES_PTRCHASE:
      if (!o.src0 || !o.dst) return set_err(CI_ERR_INVALID_ARG, "ptrchase: next and dst are required");
      if (o.n == 0 || o.n > (1ull << 32)) return set_err(CI_ERR_INVALID_ARG, "ptrchase: n must be in [1, 2^32]");
      if (o.knob != 1 && o.knob != 2 && o.knob != 4 && o.knob != 8)
        return set_err(CI_ERR_INVALID_ARG, "ptrchase: chains per lane must be 1, 2, 4 or 8");
      if ((uint64_t)grid * o.threads * o.knob >= (1ull << 31))
        return set_err(CI_ERR_INVALID_ARG, "ptrchase: too many chains");
      break;
    case CI_RES_DISPATCH:
      if (o.iters == 0 || o.iters > 0x7FFFFFFFull) return set_err(CI_ERR_INVALID_ARG, "dispatch: iters out of range");
      break;
    case CI_RES_OCCUPANCY:
      if ((uint64_t)o.knob * 1024 > 65536) return set_err(CI_ERR_INVALID_ARG, "occupancy: at most 64 KiB LDS per work-group");
      break;
    default: return set_err(CI_ERR_INVALID_ARG, "unknown resource %d", (int)r);
  }
  return CI_OK;
}

uint32_t grid_of(ci_resource_t r, const ci_stressor_opts_t& o, int ncu) {
  if (r == CI_RES_DISPATCH) return 0;
  return (uint32_t)ncu * o.wg_per_cu;
}

}  // namespace

// Workspace bytes for `ncu` CUs: control words and one record per work-group.
static size_t ws_bytes_for(ci_resource_t r, const ci_stressor_opts_t* opts, int ncu) {
  ci_stressor_opts_t o;
  resolve(r, opts, &o);
  return sizeof(DevCtrl) + (size_t)grid_of(r, o, ncu) * sizeof(ci_wg_record_t);
}

extern "C" ci_status_t ci_workspace_size(ci_resource_t r, float intensity,
                                         const ci_stressor_opts_t* opts, size_t* bytes) {
  if (!bytes || (int)r < 0 || r >= CI_RES_COUNT)
    return set_err(CI_ERR_INVALID_ARG, "ci_workspace_size: bad argument");
  if (!(intensity >= 0.0f && intensity <= 1.0f))
    return set_err(CI_ERR_INVALID_ARG, "ci_workspace_size: intensity %g not in [0, 1]", intensity);
  // the CU count of the 256-CU layout (8 XCDs x 32): exact on MI355X and an
  // upper bound on a part with fewer CUs per XCD, since the count is
  // 8 * round(per_xcd * intensity), monotone in per_xcd
  const int ncu = 8 * (int)lround(32.0 * (double)intensity);
  *bytes = ws_bytes_for(r, opts, ncu);
  return CI_OK;
}

static void wait_started(ci_stressor* h, double timeout_s) {
  const double t_end = now_s() + timeout_s;
  while (!h->ctx->host->started) {
    if (now_s() > t_end) return;
    std::this_thread::yield();
  }
}

// A persistent kernel is launched with its start event only: the end event
// is recorded when the stressor is stopped, so that while it runs nothing
// waits in its queue behind it.
static ci_status_t launch_kernel(ci_stressor* h, const KCtrl& c) {
  const ci_stressor_opts_t& o = h->o;
  hipStream_t s = h->ms;
  hipError_t e = hipSuccess;
  hipEvent_t e0 = h->e0, e1 = h->persistent ? nullptr : h->e1;
  switch (h->r) {
    case CI_RES_HBM:
    case CI_RES_MALL:
      // a read-only stream to HBM keeps fixed per-wave strides (faster there);
      // every other stream, and every Infinity-Cache stream, takes tickets
      e = launch_stream_stressor(c, o.knob, o.chunk, (const float*)o.src0, (const float*)o.src1,
                                 (float*)o.dst, o.n, o.threads, o.vec == 0, h->r == CI_RES_HBM, s, e0,
                                 e1);
      break;
    case CI_RES_L2:
    case CI_RES_VL1D: {
      const uint64_t span = cache_span_words(o);
      const uint64_t slice = 0;
      uint32_t batch = 1;
      if (!c.passes) {  // poll about every 256 KiB read per work-group
        const uint64_t b = (65536 + span - 1) / span;
        batch = (uint32_t)std::max<uint64_t>(1, b);
      }
      e = launch_cache_stressor(c, (const uint32_t*)o.src0, o.n, slice, batch, o.threads, s, e0,
                                e1);
      break;
    }
    case CI_RES_LDS:
      e = launch_lds_stressor(c, (const uint32_t*)o.src0, o.vec, o.knob, o.access == CI_LDS_LOAD, o.threads,
                              s, e0, e1);
      break;
    case CI_RES_VALU_F32:
      e = launch_valu_stressor(c, (float*)o.dst, o.knob, o.iters, o.fa, o.fb, o.threads, s, e0,
                               e1);
      break;
    case CI_RES_VALU_F64:
      e = launch_valu64_stressor(c, (double*)o.dst, o.knob, o.iters, (double)o.fa, o.threads, s,
                                 e0, e1);
      break;
    case CI_RES_MFMA_F32:
    case CI_RES_MFMA_BF16:
    case CI_RES_MFMA_FP8:
      e = launch_mfma_stressor(c, mfma_dtype(h->r), o.src0, o.src1, (float*)o.dst, o.knob, o.iters,
                               o.threads, s, e0, e1);
      break;
    case CI_RES_PTRCHASE:
      e = launch_chase_stressor(c, (const uint32_t*)o.src0, o.n, (uint32_t*)o.dst, o.knob, o.iters,
                                o.threads, s, e0, e1);
      break;
    case CI_RES_OCCUPANCY:
      e = launch_hog(c, o.knob * 1024u, o.threads, s, e0, e1);
      break;
    default: return set_err(CI_ERR_INVALID_ARG, "launch_kernel: resource %d", (int)h->r);
  }
  if (e != hipSuccess) return set_err(CI_ERR_HIP, "%s launch: %s", kResName[h->r], hipGetErrorString(e));
  return CI_OK;
}

// Dispatch stressor: a host thread keeps at most two launches of `iters`
// 64-thread work-groups in flight on the masked stream until stopped.
static void dispatch_feeder(ci_stressor* h) {
  (void)hipSetDevice(h->ctx->device);
  uint64_t* counter = h->o.dst ? (uint64_t*)h->o.dst : nullptr;
  hipEvent_t slot[2] = {h->ctx->ev[4], h->ctx->ev[5]};
  uint64_t n = 0;
  while (!h->feeder_stop.load(std::memory_order_acquire)) {
    hipEvent_t ev = slot[n & 1];
    if (n >= 2) {
      while (hipEventQuery(ev) == hipErrorNotReady) {
        if (h->feeder_stop.load(std::memory_order_acquire)) break;
        std::this_thread::yield();
      }
      if (h->feeder_stop.load(std::memory_order_acquire)) break;
    }
    hipEvent_t e0 = n == 0 ? h->e0 : nullptr;
    hipError_t e = counter ? launch_dispatch_count((uint32_t)h->o.iters, counter, h->ms, e0, nullptr)
                           : launch_dispatch_empty((uint32_t)h->o.iters, h->ms, e0, nullptr);
    if (e != hipSuccess) {
      h->feeder_err = e;
      break;
    }
    (void)hipEventRecord(ev, h->ms);
    ++n;
    h->launched.store(n, std::memory_order_release);
  }
  (void)hipEventRecord(h->e1, h->ms);
}

extern "C" ci_status_t stressor_launch(ci_ctx_t* ctx, ci_resource_t r, float intensity,
                                       void* stream, const ci_stressor_opts_t* opts, void* ws,
                                       size_t ws_bytes, ci_stressor_t** hout) {
  if (!ctx || !hout) return set_err(CI_ERR_INVALID_ARG, "stressor_launch: NULL ctx or handle");
  *hout = nullptr;
  if ((int)r < 0 || r >= CI_RES_COUNT) return set_err(CI_ERR_INVALID_ARG, "stressor_launch: resource %d", (int)r);
  if (!(intensity >= 0.0f && intensity <= 1.0f))
    return set_err(CI_ERR_INVALID_ARG, "stressor_launch: intensity %g not in [0, 1]", intensity);
  if (ctx->active) return set_err(CI_ERR_BUSY, "stressor_launch: a stressor is already running");
  if (ctx->drain_failed)
    return set_err(CI_ERR_DRAIN, "stressor_launch: an earlier stressor kernel never drained on this context");
  HIPCHK(hipSetDevice(ctx->device));
  ci_stressor* h = new (std::nothrow) ci_stressor();
  if (!h) return set_err(CI_ERR_OOM, "stressor_launch: host allocation");
  h->ctx = ctx;
  h->r = r;
  h->intensity = intensity;
  h->caller = (hipStream_t)stream;
  h->ws = ws;
  h->ws_bytes = ws_bytes;
  resolve(r, opts, &h->o);
  h->persistent = h->o.passes == 0;
  const int k = cus_for(ctx, intensity);
  h->ncu = k;
  if (k == 0) {
    h->noop = true;
    *hout = h;
    return CI_OK;
  }
  h->grid = grid_of(r, h->o, k);
  ci_status_t st = check_opts(ctx, r, h->o, h->grid);
  if (st != CI_OK) {
    delete h;
    return st;
  }
  const size_t need = ws_bytes_for(r, &h->o, k);
  if (!ws || ws_bytes < need) {
    delete h;
    return set_err(CI_ERR_INVALID_ARG, "stressor_launch: workspace %zu bytes < %zu needed", ws_bytes, need);
  }
  uint32_t mask[8];
  mask_for(ctx, k, 0, mask);
  h->ms = masked_stream(ctx, mask);
  if (!h->ms) {
    delete h;
    return set_err(CI_ERR_HIP, "hipExtStreamCreateWithCUMask failed");
  }
  h->e0 = ctx->ev[0];
  h->e1 = ctx->ev[1];
  hipError_t e = hipSuccess;
  if (h->caller) {  // a NULL caller stream is not ordered against (see coloc.h)
    e = hipEventRecord(ctx->ev[2], h->caller);
    if (e == hipSuccess) e = hipStreamWaitEvent(h->ms, ctx->ev[2], 0);
  }
  if (e == hipSuccess) e = launch_zero(ws, need, h->ms);
  if (e != hipSuccess) {
    delete h;
    return set_err(CI_ERR_HIP, "stressor_launch: stream setup: %s", hipGetErrorString(e));
  }
  ctx->host->stop = 0;
  ctx->host->started = 0;
  std::atomic_thread_fence(std::memory_order_seq_cst);

  if (r == CI_RES_DISPATCH) {
    if (h->persistent) {
      e = launch_dispatch_announce(ctx->host, h->ms);
      if (e != hipSuccess) {
        delete h;
        return set_err(CI_ERR_HIP, "dispatch announce: %s", hipGetErrorString(e));
      }
      h->feeder_stop.store(0);
      h->feeder = std::thread(dispatch_feeder, h);
      ctx->active = h;
      const double t_end = now_s() + 0.2;
      while (!ctx->host->started && now_s() < t_end) std::this_thread::yield();
    } else {
      uint64_t* counter = (uint64_t*)h->o.dst;
      for (uint64_t p = 0; p < h->o.passes; ++p) {
        hipEvent_t e0 = p == 0 ? h->e0 : nullptr;
        hipEvent_t e1 = p + 1 == h->o.passes ? h->e1 : nullptr;
        e = counter ? launch_dispatch_count((uint32_t)h->o.iters, counter, h->ms, e0, e1)
                    : launch_dispatch_empty((uint32_t)h->o.iters, h->ms, e0, e1);
        if (e != hipSuccess) {
          delete h;
          return set_err(CI_ERR_HIP, "dispatch launch: %s", hipGetErrorString(e));
        }
      }
      h->launched.store(h->o.passes);
      ctx->active = h;
    }
    *hout = h;
    return CI_OK;
  }

  KCtrl c{};
  c.host = h->persistent ? ctx->host : nullptr;
  c.dev = (DevCtrl*)ws;
  c.rec = (ci_wg_record_t*)((uint8_t*)ws + sizeof(DevCtrl));
  const uint64_t khz = (uint64_t)ctx->info.wall_clock_khz;
  c.deadline_ticks = (uint64_t)h->o.deadline_ms * khz;
  c.check_ticks = std::max<uint64_t>(1, khz / 100);   // 10 us
  c.announce_ticks = 50 * khz;                        // 50 ms
  c.passes = h->o.passes;
  c.grid = h->grid;
  c.duty = h->o.duty == 0 ? 100u : h->o.duty;
  st = launch_kernel(h, c);
  if (st != CI_OK) {
    delete h;
    return st;
  }
  ctx->active = h;
  if (h->persistent) wait_started(h, 0.25);
  *hout = h;
  return CI_OK;
}

static ci_status_t read_records(ci_ctx* ctx, const void* ws, uint32_t grid, hipStream_t s,
                                std::vector<ci_wg_record_t>& recs) {
  (void)ctx;
  recs.resize(grid);
  if (!grid) return CI_OK;
  HIPCHK(hipMemcpyAsync(recs.data(), (const uint8_t*)ws + sizeof(DevCtrl), grid * sizeof(ci_wg_record_t),
                        hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return CI_OK;
}

extern "C" ci_status_t ci_read_records(ci_ctx_t* ctx, const void* ws, uint32_t grid,
                                       ci_wg_record_t* out) {
  if (!ctx || !ws || (!out && grid)) return set_err(CI_ERR_INVALID_ARG, "ci_read_records: NULL argument");
  HIPCHK(hipSetDevice(ctx->device));
  if (!grid) return CI_OK;
  HIPCHK(hipMemcpy(out, (const uint8_t*)ws + sizeof(DevCtrl), grid * sizeof(ci_wg_record_t),
                   hipMemcpyDeviceToHost));
  return CI_OK;
}

static double units_of(const ci_stressor* h, const std::vector<ci_wg_record_t>& recs,
                       uint64_t work) {
  const ci_stressor_opts_t& o = h->o;
  const double waves = o.threads / 64.0;
  switch (h->r) {
    case CI_RES_HBM:
    case CI_RES_MALL: {
      const double per = hbm_bytes_per_element(o.knob);
      if (!h->persistent) return per * (double)o.n * (double)o.passes;
      return per * 256.0 * o.chunk * (double)work;  // whole wave-chunks (the ragged last one counted full)
    }
    case CI_RES_L2:
    case CI_RES_VL1D:
      return 4.0 * (double)cache_span_words(o) * (double)work;
    case CI_RES_LDS:  // every lane walks the 8192-word window once per pass: loads, plus stores for copy
      return (double)work * waves * 64.0 * 8192.0 * 4.0 * (o.access == CI_LDS_LOAD ? 1.0 : 2.0);
    case CI_RES_VALU_F32: return (double)work * o.threads * o.knob * (double)o.iters * 2.0;
    case CI_RES_MFMA_F32:
    case CI_RES_MFMA_BF16:
    case CI_RES_MFMA_FP8:
      return (double)work * waves * o.knob * (double)o.iters * 2.0 * 32 * 32 * mfma_k(mfma_dtype(h->r));
    case CI_RES_PTRCHASE: return (double)work * o.threads * o.knob * (double)o.iters;
    case CI_RES_VALU_F64: return (double)work * o.threads * o.knob * (double)o.iters;
    case CI_RES_DISPATCH: return (double)h->launched.load() * (double)o.iters;
    default: return 0.0;
  }
  (void)recs;
}

extern "C" ci_status_t stressor_stop(ci_stressor_t* h, ci_stressor_report_t* rep) {
  if (!h) return set_err(CI_ERR_INVALID_ARG, "stressor_stop: NULL handle");
  ci_ctx* ctx = h->ctx;
  if (rep) {
    memset(rep, 0, sizeof(*rep));
    rep->resource = h->r;
    rep->ncu = h->ncu;
    rep->grid = h->grid;
  }
  if (h->noop) {
    delete h;
    return CI_OK;
  }
  (void)hipSetDevice(ctx->device);
  ctx->host->stop = 1;
  std::atomic_thread_fence(std::memory_order_seq_cst);
  if (h->feeder.joinable()) {
    h->feeder_stop.store(1, std::memory_order_release);
    h->feeder.join();
  } else if (h->persistent) {
    // the end event of a persistent kernel is queued only now
    hipError_t er = hipEventRecord(h->e1, h->ms);
    if (er != hipSuccess) {
      (void)hipStreamSynchronize(h->ms);
      ctx->active = nullptr;
      delete h;
      return set_err(CI_ERR_HIP, "stressor_stop: end event: %s", hipGetErrorString(er));
    }
  }
  // Drain: every wave exits on the flag or on its own deadline.
  const double limit = now_s() + h->o.deadline_ms * 1e-3 + 5.0;
  hipError_t q;
  while ((q = hipEventQuery(h->e1)) == hipErrorNotReady && now_s() < limit)
    std::this_thread::sleep_for(std::chrono::microseconds(20));
  ci_status_t st = CI_OK;
  if (q == hipErrorNotReady) {
    // The kernel may still be running and polling the stop word, which stays
    // raised: the context refuses further stressors (a new launch would
    // clear the word and let the old kernel overlap later runs).
    ctx->drain_failed = true;
    ctx->active = nullptr;
    delete h;
    return set_err(CI_ERR_DRAIN, "stressor_stop: kernel did not drain within its deadline + 5 s");
  }
  hipError_t e = hipStreamSynchronize(h->ms);
  if (e != hipSuccess) st = set_err(CI_ERR_HIP, "stressor kernel: %s", hipGetErrorString(e));
  if (st == CI_OK && h->caller) {
    e = hipEventRecord(ctx->ev[3], h->ms);
    if (e == hipSuccess) e = hipStreamWaitEvent(h->caller, ctx->ev[3], 0);
    if (e != hipSuccess) st = set_err(CI_ERR_HIP, "stressor_stop: stream join: %s", hipGetErrorString(e));
  }
  float ms = 0.0f;
  if (st == CI_OK && hipEventElapsedTime(&ms, h->e0, h->e1) != hipSuccess) ms = 0.0f;
  std::vector<ci_wg_record_t> recs;
  if (st == CI_OK) st = read_records(ctx, h->ws, h->grid, h->ms, recs);
  if (st == CI_OK && h->feeder_err != hipSuccess)
    st = set_err(CI_ERR_HIP, "dispatch feeder: %s", hipGetErrorString(h->feeder_err));
  if (st == CI_OK && rep) {
    uint64_t work = 0, chk = 0, fs = UINT64_MAX, ls = 0, fe = UINT64_MAX, le = 0;
    uint32_t reported = 0;
    int timed_out = 0;
    std::vector<uint32_t> locs;
    for (const auto& rc : recs) {
      if (rc.t_end == 0) continue;
      ++reported;
      work += rc.work;
      chk += rc.check;
      fs = std::min(fs, rc.t_start);
      ls = std::max(ls, rc.t_start);
      fe = std::min(fe, rc.t_end);
      le = std::max(le, rc.t_end);
      if (rc.flags & kRecFlagDeadline) timed_out = 1;
      locs.push_back(rc.loc);
    }
    std::sort(locs.begin(), locs.end());
    rep->distinct_cus = (int)(std::unique(locs.begin(), locs.end()) - locs.begin());
    rep->wg_reported = reported;
    rep->work = work;
    rep->checksum = chk;
    rep->timed_out = timed_out;
    rep->kernel_ns = (double)ms * 1e6;
    const double tick_ns = 1e6 / (double)ctx->info.wall_clock_khz;
    if (reported) {
      rep->t_first_start = fs;
      rep->t_last_start = ls;
      rep->t_first_end = fe;
      rep->t_last_end = le;
      rep->window_ns = (double)(le - fs) * tick_ns;
    } else {
      rep->window_ns = rep->kernel_ns;
    }
    rep->units = units_of(h, recs, work);
    const double secs = (h->persistent ? rep->window_ns : rep->kernel_ns) * 1e-9;
    rep->achieved = secs > 0 ? rep->units / secs : 0.0;
    const double pk = ctx->info.peak[h->r];
    rep->pct_of_peak = pk > 0 ? 100.0 * rep->achieved / pk : 0.0;
    if (timed_out) st = set_err(CI_ERR_TIMEOUT, "%s: work-groups stopped on their deadline", kResName[h->r]);
  }
  ctx->active = nullptr;
  delete h;
  return st;
}

// ------------------------------------------------------- queue-pair check
// Kernels on two hardware queues can slow each other although they share no
// CU and no memory traffic: on MI355X a victim beside a sleeping kernel on
// another queue ran either at its alone speed or 1.4-1.6x slower, depending
// only on the order in which the process had created its queues (in three
// of six random orders; the sleeping kernel's shape made no difference).
// Before the first colocated measurement of a (victim queue, stressor
// queue) pair in a measurement call (one victim), the victim therefore runs
// alone and beside an idle kernel on the stressor's queue, in
// counterbalanced order; if the idle kernel alone slows it by more than
// kQueueTol, a queue is replaced (the stressor's and the victim's in turn)
// and the check repeated, kQueueAttempts times at most.  The idle kernel is
// one 256-thread work-group per stressed CU on shared CUs (most wave slots
// stay free for the victim) and takes the stressor's shape (threads,
// work-groups per CU) on disjoint CUs.
namespace {
constexpr double kQueueTol = 1.05;
constexpr int kQueueAttempts = 8;
constexpr int kQueuePairs = 6;

// Replaces the shared-placement victim stream (a plain stream: the runtime
// deals plain streams round-robin over its hardware queues).
hipStream_t new_plain_stream(ci_ctx* ctx) {
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
  ++ctx->queue_gen;
  return s;
}

hipStream_t replace_vstream(ci_ctx* ctx) {
  hipStream_t s = new_plain_stream(ctx);
  if (!s) return nullptr;
  destroy_stream(ctx, ctx->vstream);
  ctx->vstream = s;
  return s;
}

ci_status_t median_alone(hipStream_t s, ci_status_t (*run)(void*, hipStream_t, double*), void* arg,
                         double* out) {
  std::vector<double> t;
  for (int i = 0; i < 2 + kQueuePairs; ++i) {
    double ns = 0.0;
    const ci_status_t st = run(arg, s, &ns);
    if (st != CI_OK) return st;
    if (i >= 2) t.push_back(ns);
  }
  *out = median(t);
  return CI_OK;
}

// A victim queue can also be slow on its own: the same kernel alone on two
// queues with the same CU mask has run 1.5x apart.  Before its first pair
// check in a measurement call, the victim's queue is measured against
// kQualifyCandidates freshly created queues with the same mask (created
// while the others exist, so they land elsewhere), and the fastest is kept.
constexpr int kQualifyCandidates = 2;
constexpr double kQualifyGain = 0.97;

ci_status_t qualify_victim_queue(ci_ctx* ctx, hipStream_t* vs, const uint32_t* vmask,
                                 ci_status_t (*run)(void*, hipStream_t, double*), void* arg) {
  for (const auto& q : ctx->queue_qualified)
    if (q.first == *vs && q.second == ctx->queue_gen) return CI_OK;
  std::array<uint32_t, 8> key{};
  if (vmask)
    for (int i = 0; i < 8; ++i) key[i] = vmask[i];
  hipStream_t best = *vs;
  double t_best = 0.0;
  ci_status_t st = median_alone(best, run, arg, &t_best);
  if (st != CI_OK) return st;
  for (int c = 0; c < kQualifyCandidates; ++c) {
    hipStream_t cand = vmask ? new_masked_stream(ctx, key) : new_plain_stream(ctx);
    if (!cand) return set_err(CI_ERR_HIP, "victim queue qualification: stream creation failed");
    double t = 0.0;
    st = median_alone(cand, run, arg, &t);
    hipStream_t loser = cand;
    if (st == CI_OK && t < kQualifyGain * t_best) {
      loser = best;
      best = cand;
      t_best = t;
    }
    if (loser != *vs) destroy_stream(ctx, loser);
    if (st != CI_OK) return st;
  }
  if (best != *vs) {  // install the winner where the old victim queue was kept
    ++ctx->queue_replaced;
    destroy_stream(ctx, *vs);
    if (vmask) {
      ctx->masked[key] = best;
      ctx->masked_used[key] = ++ctx->use_clock;
    } else {
      ctx->vstream = best;
    }
    *vs = best;
  }
  ctx->queue_qualified.push_back({best, ctx->queue_gen});
  return CI_OK;
}
}  // namespace

ci_status_t ci::check_queue_pair(ci_ctx* ctx, ci_resource_t r, const ci_stressor_opts_t* so,
                                 float intensity, hipStream_t caller, hipStream_t* vs,
                                 const uint32_t* vmask, void* ws, size_t ws_bytes,
                                 ci_status_t (*run)(void*, hipStream_t, double*), void* arg,
                                 int* unresolved) {
  if (unresolved) *unresolved = 0;
  const int k = cus_for(ctx, intensity);
  if (k == 0) return CI_OK;
  uint32_t mask[8];
  mask_for(ctx, k, 0, mask);
  hipStream_t ss = masked_stream(ctx, mask);
  if (!ss) return set_err(CI_ERR_HIP, "hipExtStreamCreateWithCUMask failed");
  ci_stressor_opts_t o{};
  o.threads = 256;  // shared CUs: one 256-thread work-group per CU
  o.wg_per_cu = 1;
  if (vmask) {  // disjoint CUs: the stressor's own launch shape
    ci_stressor_opts_t ro;
    resolve(r, so, &ro);
    o.threads = ro.threads ? ro.threads : 64;
    o.wg_per_cu = ro.wg_per_cu ? ro.wg_per_cu : 1;
    if ((uint64_t)o.wg_per_cu * o.threads > 2048) o.wg_per_cu = 2048 / o.threads;
  }
  o.knob = 1;  // 1 KiB of LDS
  o.deadline_ms = 1000;
  ci_status_t qs = qualify_victim_queue(ctx, vs, vmask, run, arg);
  if (qs != CI_OK) return qs;
  for (const auto& p : ctx->queue_checked)
    if (p.victim == *vs && p.stressor == ss && p.threads == o.threads && p.wg_per_cu == o.wg_per_cu &&
        p.gen == ctx->queue_gen) {
      if (unresolved) *unresolved = p.unresolved;
      return CI_OK;
    }
  const size_t need = ws_bytes_for(CI_RES_OCCUPANCY, &o, k);
  if (!ws || ws_bytes < need) return CI_OK;  // no room for the idle kernel: the pair stays unchecked
  ++ctx->queue_checks;
  int unres = 0;
  for (int attempt = 0;; ++attempt) {
    ci_status_t st = CI_OK;
    double t = 0.0;
    for (int w = 0; w < 2 && st == CI_OK; ++w) st = run(arg, *vs, &t);
    if (st != CI_OK) return st;
    std::vector<double> ta, ti;
    for (int rep = 0; rep < kQueuePairs; ++rep) {
      const bool idle_first = rep & 1;
      double t_alone = 0.0, t_idle = 0.0;
      if (!idle_first && (st = run(arg, *vs, &t_alone)) != CI_OK) return st;
      ci_stressor_t* h = nullptr;
      st = stressor_launch(ctx, CI_RES_OCCUPANCY, intensity, caller, &o, ws, ws_bytes, &h);
      if (st != CI_OK) return st;
      const ci_status_t vst = run(arg, *vs, &t_idle);
      st = stressor_stop(h, nullptr);
      if (vst != CI_OK) return vst;
      if (st != CI_OK) return st;
      if (idle_first && (st = run(arg, *vs, &t_alone)) != CI_OK) return st;
      ta.push_back(t_alone);
      ti.push_back(t_idle);
    }
    if (median(ti) <= kQueueTol * median(ta)) break;
    if (attempt + 1 >= kQueueAttempts) {  // measured as placed; not retried
      ++ctx->queue_unresolved;
      unres = 1;
      break;
    }
    ++ctx->queue_replaced;
    if (attempt % 2 == 0) {
      ss = replace_masked_stream(ctx, mask);
      if (!ss) return set_err(CI_ERR_HIP, "hipExtStreamCreateWithCUMask failed");
    } else {
      hipStream_t nv = vmask ? replace_masked_stream(ctx, vmask) : replace_vstream(ctx);
      if (!nv) return set_err(CI_ERR_HIP, "victim stream replacement failed");
      *vs = nv;
      qs = qualify_victim_queue(ctx, vs, vmask, run, arg);
      if (qs != CI_OK) return qs;
    }
  }
  ctx->queue_checked.push_back({*vs, ss, o.threads, o.wg_per_cu, ctx->queue_gen, unres});
  if (unresolved) *unresolved = unres;
  return CI_OK;
}

extern "C" ci_status_t ci_queue_stats(ci_ctx_t* ctx, uint32_t* checks, uint32_t* replaced,
                                      uint32_t* unresolved) {
  if (!ctx || !checks || !replaced || !unresolved)
    return set_err(CI_ERR_INVALID_ARG, "ci_queue_stats: NULL argument");
  *checks = ctx->queue_checks;
  *replaced = ctx->queue_replaced;
  *unresolved = ctx->queue_unresolved;
  return CI_OK;
}

// ------------------------------------------------------------------ victims
namespace {

ci_status_t check_victim(const ci_victim_desc_t* d) {
  if (!d) return set_err(CI_ERR_INVALID_ARG, "victim: NULL descriptor");
  if (d->reserved) return set_err(CI_ERR_INVALID_ARG, "victim: reserved field must be 0");
  if (d->flags & ~(d->kind == CI_VICTIM_TRIAD_F32 ? CI_VICTIM_TRIAD_IN_KERNEL : 0u))
    return set_err(CI_ERR_INVALID_ARG, "victim: flags 0x%x not valid for kind %d", d->flags, d->kind);
  switch (d->kind) {
    case CI_VICTIM_TRIAD_F32:
      if (d->n && (!d->a || !d->b || !d->out)) return set_err(CI_ERR_INVALID_ARG, "triad: NULL operand");
      if (((uintptr_t)d->a | (uintptr_t)d->b | (uintptr_t)d->out) & 15)
        return set_err(CI_ERR_INVALID_ARG, "triad: arrays must be 16-byte aligned");
      if (d->passes == 0) return set_err(CI_ERR_INVALID_ARG, "triad: passes must be >= 1");
      return CI_OK;
    case CI_VICTIM_GEMM: {
      if (d->dtype != CI_DT_F32 && d->dtype != CI_DT_BF16 && d->dtype != CI_DT_FP8E4M3)
        return set_err(CI_ERR_INVALID_ARG, "gemm: dtype %d", d->dtype);
      const uint64_t es = d->dtype == CI_DT_F32 ? 4 : d->dtype == CI_DT_BF16 ? 2 : 1;
      if (d->m == 0 || d->n == 0 || d->k == 0) return set_err(CI_ERR_INVALID_ARG, "gemm: empty shape");
      if ((d->k * es) % 16) return set_err(CI_ERR_INVALID_ARG, "gemm: K*elem must be a multiple of 16 bytes");
      if (d->m > 0xFFFFFF80ull || d->n > 0xFFFFFF80ull || d->k > 0x0FFFFFFFull)
        return set_err(CI_ERR_INVALID_ARG, "gemm: shape too large");
      if (!d->a || !d->b || !d->out) return set_err(CI_ERR_INVALID_ARG, "gemm: NULL operand");
      if (((uintptr_t)d->a | (uintptr_t)d->b) & 15) return set_err(CI_ERR_INVALID_ARG, "gemm: A and B must be 16-byte aligned");
      if (((d->m + 127) / 128) * ((d->n + 127) / 128) > 0x7FFFFFFFull)
        return set_err(CI_ERR_INVALID_ARG, "gemm: too many tiles");
      return CI_OK;
    }
    case CI_VICTIM_GEMV:
      if (d->dtype != CI_DT_BF16) return set_err(CI_ERR_INVALID_ARG, "gemv: only BF16 weights");
      if (d->n == 0 || d->k == 0 || d->k % 8) return set_err(CI_ERR_INVALID_ARG, "gemv: k must be a positive multiple of 8");
      if (!d->a || !d->b || !d->out) return set_err(CI_ERR_INVALID_ARG, "gemv: NULL operand");
      if (((uintptr_t)d->a | (uintptr_t)d->b) & 15) return set_err(CI_ERR_INVALID_ARG, "gemv: W and x must be 16-byte aligned");
      if (d->copies == 0) return set_err(CI_ERR_INVALID_ARG, "gemv: copies must be >= 1");
      return CI_OK;
    default: return set_err(CI_ERR_INVALID_ARG, "victim: kind %d", d->kind);
  }
}

uint64_t victim_out_len(const ci_victim_desc_t* d) {
  switch (d->kind) {
    case CI_VICTIM_TRIAD_F32: return d->n;
    case CI_VICTIM_GEMM: return d->m * d->n;
    default: return d->n;
  }
}

}  // namespace

ci_status_t ci::launch_victim(ci_ctx* ctx, const ci_victim_desc_t* d, hipStream_t s, hipEvent_t e0,
                              hipEvent_t e1) {
  hipError_t e = hipSuccess;
  switch (d->kind) {
    case CI_VICTIM_TRIAD_F32: {
      if (d->n == 0) {
        if (e0) e = hipEventRecord(e0, s);
        if (e == hipSuccess && e1) e = hipEventRecord(e1, s);
        break;
      }
      uint64_t g = (d->n + 4095) / 4096;
      const uint64_t cap = (uint64_t)ctx->info.num_cus * 8;
      if (g > cap) g = cap;
      e = launch_triad_victim((const float*)d->a, (const float*)d->b, (float*)d->out, d->n, d->passes,
                              (d->flags & CI_VICTIM_TRIAD_IN_KERNEL) != 0, (uint32_t)g, s, e0, e1);
      break;
    }
    case CI_VICTIM_GEMM: {
      const float scale = d->dtype == CI_DT_FP8E4M3 ? d->scale_a * d->scale_b : 1.0f;
      e = launch_gemm(d->dtype, d->a, d->b, (float*)d->out, d->m, d->n, d->k, scale, s, e0, e1);
      break;
    }
    case CI_VICTIM_GEMV: {
      const uint64_t copy = ctx->rot++ % d->copies;
      const uint16_t* w = (const uint16_t*)d->a + copy * d->n * d->k;
      e = launch_gemv_bf16(w, (const uint16_t*)d->b, (float*)d->out, d->n, d->k, s, e0, e1);
      break;
    }
    default: return set_err(CI_ERR_INVALID_ARG, "victim kind %d", d->kind);
  }
  if (e != hipSuccess) return set_err(CI_ERR_HIP, "victim launch: %s", hipGetErrorString(e));
  return CI_OK;
}

// Run one victim on exec stream `xs` after the caller's queued work; fills
// out (time, stamps, checksums).  Blocks until done.
ci_status_t ci::run_victim(ci_ctx* ctx, const ci_victim_desc_t* d, hipStream_t caller, hipStream_t xs,
                           ci_victim_result_t* out) {
  volatile uint64_t* hr = ctx->hres;
  hr[0] = hr[1] = hr[2] = hr[3] = 0;
  if (caller) {
    HIPCHK(hipEventRecord(ctx->ev[6], caller));
    HIPCHK(hipStreamWaitEvent(xs, ctx->ev[6], 0));
  }
  HIPCHK(launch_stamp((uint64_t*)&hr[0], xs));
  ci_status_t st = launch_victim(ctx, d, xs, ctx->ev[7], ctx->ev[8]);
  if (st != CI_OK) return st;
  HIPCHK(launch_stamp((uint64_t*)&hr[1], xs));
  const uint64_t len = victim_out_len(d);
  HIPCHK(launch_checksum_f32((const float*)d->out, len, ctx->part_bits, ctx->part_sum, ctx->nparts,
                             (uint64_t*)&hr[2], (double*)&hr[3], xs));
  HIPCHK(hipEventRecord(ctx->ev[9], xs));
  if (caller) HIPCHK(hipStreamWaitEvent(caller, ctx->ev[9], 0));
  HIPCHK(hipEventSynchronize(ctx->ev[9]));
  float ms = 0.0f;
  HIPCHK(hipEventElapsedTime(&ms, ctx->ev[7], ctx->ev[8]));
  out->time_ns = (double)ms * 1e6;
  out->t_begin = hr[0];
  out->t_end = hr[1];
  out->checksum_bits = hr[2];
  uint64_t sb = hr[3];
  memcpy(&out->sum_f64, &sb, sizeof(double));
  return CI_OK;
}

extern "C" ci_status_t victim_run(ci_ctx_t* ctx, const ci_victim_desc_t* d, void* stream,
                                  ci_victim_result_t* out) {
  if (!ctx || !out) return set_err(CI_ERR_INVALID_ARG, "victim_run: NULL argument");
  ci_status_t st = check_victim(d);
  if (st != CI_OK) return st;
  HIPCHK(hipSetDevice(ctx->device));
  return run_victim(ctx, d, (hipStream_t)stream, ctx->vstream, out);
}

extern "C" ci_status_t victim_enqueue(ci_ctx_t* ctx, const ci_victim_desc_t* d, void* stream,
                                      uint32_t count) {
  if (!ctx || !stream) return set_err(CI_ERR_INVALID_ARG, "victim_enqueue: NULL ctx or stream");
  ci_status_t st = check_victim(d);
  if (st != CI_OK) return st;
  HIPCHK(hipSetDevice(ctx->device));
  for (uint32_t i = 0; i < count; ++i) {
    st = launch_victim(ctx, d, (hipStream_t)stream, nullptr, nullptr);
    if (st != CI_OK) return st;
  }
  return CI_OK;
}

extern "C" ci_status_t ci_stamp(ci_ctx_t* ctx, uint64_t* slot, void* stream) {
  if (!ctx || !slot || !stream) return set_err(CI_ERR_INVALID_ARG, "ci_stamp: NULL argument");
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(launch_stamp(slot, (hipStream_t)stream));
  return CI_OK;
}

extern "C" ci_status_t ci_checksum_f32(ci_ctx_t* ctx, const void* x, uint64_t n, void* stream,
                                       uint64_t* bits, double* sum) {
  if (!ctx || (!x && n) || !bits || !sum) return set_err(CI_ERR_INVALID_ARG, "ci_checksum_f32: NULL argument");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  volatile uint64_t* hr = ctx->hres;
  HIPCHK(launch_checksum_f32((const float*)x, n, ctx->part_bits, ctx->part_sum, ctx->nparts,
                             (uint64_t*)&hr[4], (double*)&hr[5], s));
  HIPCHK(hipStreamSynchronize(s));
  *bits = hr[4];
  uint64_t sb = hr[5];
  memcpy(sum, &sb, sizeof(double));
  return CI_OK;
}

extern "C" ci_status_t ci_mfma_probe(ci_ctx_t* ctx, int dtype, const void* a, const void* b,
                                     const float* c, float* d, uint32_t ntiles, void* stream) {
  if (!ctx || (ntiles && (!a || !b || !c || !d)))
    return set_err(CI_ERR_INVALID_ARG, "ci_mfma_probe: NULL argument");
  if (dtype != CI_DT_F32 && dtype != CI_DT_BF16 && dtype != CI_DT_FP8E4M3)
    return set_err(CI_ERR_INVALID_ARG, "ci_mfma_probe: dtype %d", dtype);
  if (ntiles == 0) return CI_OK;
  if (ntiles > 0x7FFFFFFFu) return set_err(CI_ERR_INVALID_ARG, "ci_mfma_probe: too many tiles");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(launch_mfma_probe(dtype, a, b, c, d, ntiles, s));
  HIPCHK(hipStreamSynchronize(s));
  return CI_OK;
}

extern "C" ci_status_t ci_quantize(ci_ctx_t* ctx, const void* src, uint64_t n, int dtype, void* dst,
                                   float* scale_out, void* stream) {
  if (!ctx || (n && (!src || !dst))) return set_err(CI_ERR_INVALID_ARG, "ci_quantize: NULL argument");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  if (dtype == CI_DT_BF16) {
    HIPCHK(launch_to_bf16((const float*)src, n, (uint16_t*)dst, s));
    HIPCHK(hipStreamSynchronize(s));
    if (scale_out) *scale_out = 1.0f;
    return CI_OK;
  }
  if (dtype != CI_DT_FP8E4M3) return set_err(CI_ERR_INVALID_ARG, "ci_quantize: dtype %d", dtype);
  HIPCHK(launch_amax_f32((const float*)src, n, ctx->amax_part, ctx->nparts, ctx->amax_out, s));
  HIPCHK(launch_to_fp8((const float*)src, n, ctx->amax_out, (uint8_t*)dst, s));
  float amax = 0.0f;
  HIPCHK(hipMemcpyAsync(&amax, ctx->amax_out, sizeof(float), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (scale_out) {
    volatile float m = amax, q = 448.0f;
    *scale_out = (amax > 0.0f && std::isfinite(amax)) ? (float)(m / q) : 1.0f;
  }
  return CI_OK;
}

// -------------------------------------------------------------- sensitivity
double ci::median(std::vector<double> v) {
  if (v.empty()) return NAN;
  std::sort(v.begin(), v.end());
  const size_t n = v.size();
  return n % 2 ? v[n / 2] : 0.5 * (v[n / 2 - 1] + v[n / 2]);
}

double ci::quantile(std::vector<double> v, double q) {
  if (v.empty()) return NAN;
  std::sort(v.begin(), v.end());
  const double pos = q * (double)(v.size() - 1);
  const size_t lo = (size_t)std::floor(pos), hi = (size_t)std::ceil(pos);
  return v[lo] + (v[hi] - v[lo]) * (pos - (double)lo);
}


namespace {
uint64_t sm64_word(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
}  // namespace

extern "C" ci_status_t ci_bootstrap_slowdown(const double* alone, uint32_t na, const double* col,
                                             uint32_t nc, uint32_t resamples, uint64_t seed,
                                             double* lo, double* hi) {
  if (!alone || !col || !lo || !hi || na == 0 || nc == 0 || resamples == 0)
    return set_err(CI_ERR_INVALID_ARG, "ci_bootstrap_slowdown: NULL pointer or zero count");
  std::vector<double> ratios(resamples), ra(na), rc(nc);
  for (uint32_t r = 0; r < resamples; ++r) {
    const uint64_t k0 = (uint64_t)r * ((uint64_t)na + nc);
    for (uint32_t j = 0; j < na; ++j) ra[j] = alone[sm64_word(seed, k0 + j) % na];
    for (uint32_t j = 0; j < nc; ++j) rc[j] = col[sm64_word(seed, k0 + na + j) % nc];
    ratios[r] = median(rc) / median(ra);
  }
  *lo = quantile(ratios, 0.025);
  *hi = quantile(ratios, 0.975);
  return CI_OK;
}

namespace {
struct VictimRun {
  ci_ctx* ctx;
  const ci_victim_desc_t* d;
  hipStream_t caller;
  static ci_status_t call(void* p, hipStream_t vs, double* ns) {
    VictimRun* v = static_cast<VictimRun*>(p);
    ci_victim_result_t r;
    const ci_status_t st = run_victim(v->ctx, v->d, v->caller, vs, &r);
    *ns = r.time_ns;
    return st;
  }
};
}  // namespace

extern "C" ci_status_t measure_sensitivity(ci_ctx_t* ctx, const ci_victim_desc_t* d,
                                           const ci_resource_t* rs, const ci_stressor_opts_t* sopts,
                                           int nr, const float* xs, int nx,
                                           const ci_measure_opts_t* o, void* ws, size_t ws_bytes,
                                           void* stream, ci_cell_t* cells) {
  if (!ctx || !rs || !xs || !cells || nr <= 0 || nx <= 0)
    return set_err(CI_ERR_INVALID_ARG, "measure_sensitivity: bad argument");
  ci_status_t st = check_victim(d);
  if (st != CI_OK) return st;
  ci_measure_opts_t mo{};
  mo.reps = 20;
  mo.warmups = 3;
  mo.placement = CI_PLACE_SHARED;
  mo.deadline_ms = 2000;
  if (o) {
    mo = *o;
    if (!mo.reps) mo.reps = 20;
    if (!mo.deadline_ms) mo.deadline_ms = 2000;
  }
  for (int j = 0; j < nx; ++j)
    if (!(xs[j] >= 0.0f && xs[j] <= 1.0f))
      return set_err(CI_ERR_INVALID_ARG, "measure_sensitivity: intensity %g", xs[j]);
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t caller = (hipStream_t)stream;
  ctx->queue_checked.clear();  // queue pairs are checked per victim
  ctx->queue_qualified.clear();
  // per-rep times of cell c, rep r at index c * reps + r (NaN where a cell
  // is not measured)
  if (mo.rep_alone_ns || mo.rep_col_ns)
    for (size_t q = 0; q < (size_t)nr * nx * mo.reps; ++q) {
      if (mo.rep_alone_ns) mo.rep_alone_ns[q] = NAN;
      if (mo.rep_col_ns) mo.rep_col_ns[q] = NAN;
    }
  for (int i = 0; i < nr; ++i) {
    for (int j = 0; j < nx; ++j) {
      ci_cell_t& cell = cells[i * nx + j];
      const size_t rep0 = (size_t)(i * nx + j) * mo.reps;
      memset(&cell, 0, sizeof(cell));
      cell.resource = rs[i];
      cell.intensity = xs[j];
      const int k = cus_for(ctx, xs[j]);
      cell.ncu = k;
      hipStream_t vs = ctx->vstream;
      HeldStream hold(ctx, &vs);  // the cache never evicts the victim's stream
      uint32_t vmask[8];
      const bool masked = mo.placement == CI_PLACE_DISJOINT && k > 0;  // k == 0: whole GPU, unmasked
      if (masked) {
        if (k >= ctx->info.num_cus) {  // no CUs left for the victim
          cell.slowdown = cell.slowdown_p10 = cell.slowdown_p90 = NAN;
          cell.slowdown_ci_lo = cell.slowdown_ci_hi = NAN;
          continue;
        }
        mask_for(ctx, k, 1, vmask);
        vs = masked_stream(ctx, vmask);
        if (!vs) return set_err(CI_ERR_HIP, "hipExtStreamCreateWithCUMask failed");
      }
      ci_stressor_opts_t so{};
      if (sopts) so = sopts[i];
      so.passes = 0;
      so.deadline_ms = mo.deadline_ms;
      ci_victim_result_t r;
      VictimRun vr{ctx, d, caller};
      if (!(mo.flags & CI_MEASURE_NO_QUEUE_CHECK)) {
        st = check_queue_pair(ctx, rs[i], sopts ? &sopts[i] : nullptr, xs[j], caller, &vs,
                              masked ? vmask : nullptr, ws, ws_bytes, &VictimRun::call, &vr,
                              &cell.queue_unresolved);
        if (st != CI_OK) return st;
      }
      for (uint32_t w = 0; w < mo.warmups; ++w) {
        st = run_victim(ctx, d, caller, vs, &r);
        if (st != CI_OK) return st;
      }
      std::vector<double> ta, tc, ratio;
      double ach = 0.0, pct = 0.0;
      int covered = 1, equal = 1, timed = 0, nrep = 0;
      for (uint32_t rep = 0; rep < mo.reps; ++rep) {
        // counterbalanced order (alone, colocated, colocated, alone, ...):
        // drift and carry-over from the previous run (clock, caches the
        // stressor left cold) fall on both sides equally
        const bool col_first = rep & 1u;
        ci_victim_result_t ra, rc;
        if (!col_first) {
          st = run_victim(ctx, d, caller, vs, &ra);
          if (st != CI_OK) return st;
        }
        ci_stressor_t* h = nullptr;
        st = stressor_launch(ctx, rs[i], xs[j], caller, &so, ws, ws_bytes, &h);
        if (st != CI_OK) return st;
        ci_status_t vst = run_victim(ctx, d, caller, vs, &rc);
        ci_stressor_report_t sr;
        const bool noop = h->noop;
        st = stressor_stop(h, &sr);
        if (vst != CI_OK) return vst;
        if (st == CI_ERR_TIMEOUT) {
          timed = 1;
        } else if (st != CI_OK) {
          return st;
        }
        if (col_first) {
          st = run_victim(ctx, d, caller, vs, &ra);
          if (st != CI_OK) return st;
        }
        if (!noop && rs[i] != CI_RES_DISPATCH) {
          if (!(sr.t_last_start <= rc.t_begin && sr.t_first_end >= rc.t_end) ||
              sr.wg_reported != sr.grid)
            covered = 0;
        }
        if (rc.checksum_bits != ra.checksum_bits) equal = 0;
        if (mo.rep_alone_ns) mo.rep_alone_ns[rep0 + rep] = ra.time_ns;
        if (mo.rep_col_ns) mo.rep_col_ns[rep0 + rep] = rc.time_ns;
        ta.push_back(ra.time_ns);
        tc.push_back(rc.time_ns);
        ratio.push_back(rc.time_ns / ra.time_ns);
        ach += sr.achieved;
        pct += sr.pct_of_peak;
        ++nrep;
      }
      cell.reps = nrep;
      cell.t_alone_ns = median(ta);
      cell.t_col_ns = median(tc);
      cell.slowdown = cell.t_col_ns / cell.t_alone_ns;
      cell.slowdown_p10 = quantile(ratio, 0.1);
      cell.slowdown_p90 = quantile(ratio, 0.9);
      cell.slowdown_ci_lo = cell.slowdown_ci_hi = NAN;
      if (nrep)
        (void)ci_bootstrap_slowdown(ta.data(), (uint32_t)ta.size(), tc.data(), (uint32_t)tc.size(),
                                    1000, 16909ull + (uint64_t)(&cell - cells), &cell.slowdown_ci_lo,
                                    &cell.slowdown_ci_hi);
      cell.stressor_achieved = nrep ? ach / nrep : 0.0;
      cell.stressor_pct_peak = nrep ? pct / nrep : 0.0;
      cell.window_covered = covered;
      cell.output_equal = equal;
      cell.timed_out = timed;
    }
  }
  return CI_OK;
}
