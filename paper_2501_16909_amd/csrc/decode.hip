// Host runtime of the synthetic decode step: config validation and layouts,
// the step itself (one timed launch per kernel), the kernels one at a time,
// and the step's sensitivity measurement beside a stressor.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"
#include "runtime.h"

using namespace ci;

namespace {

constexpr uint32_t kChunk = 64;   // attention positions per work-group

uint64_t al64(uint64_t x) { return (x + 63) & ~63ull; }
size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Work {
  size_t x, xn, qkv, qrot, part, attn, gu, h, total;
  uint32_t nchunks;
};

ci_status_t check_cfg(const ci_decode_config_t* c) {
  if (!c) return set_err(CI_ERR_INVALID_ARG, "decode: NULL config");
  if (c->hidden == 0 || c->hidden % 8) return set_err(CI_ERR_INVALID_ARG, "decode: hidden %u must be a positive multiple of 8", c->hidden);
  if (c->ffn == 0 || c->ffn % 8) return set_err(CI_ERR_INVALID_ARG, "decode: ffn %u must be a positive multiple of 8", c->ffn);
  if (c->head_dim != 128 && c->head_dim != 256) return set_err(CI_ERR_INVALID_ARG, "decode: head_dim %u not 128 or 256", c->head_dim);
  if (c->n_kv == 0 || c->n_q == 0 || c->n_q % c->n_kv || c->n_q / c->n_kv > 16)
    return set_err(CI_ERR_INVALID_ARG, "decode: n_q %u / n_kv %u must be a whole group of 1..16", c->n_q, c->n_kv);
  if (c->layers == 0) return set_err(CI_ERR_INVALID_ARG, "decode: layers must be >= 1");
  if (c->batch == 0 || c->batch > kDecodeMaxBatch) return set_err(CI_ERR_INVALID_ARG, "decode: batch %u not in 1..%u", c->batch, kDecodeMaxBatch);
  if (c->max_ctx == 0 || c->max_ctx > (1u << 24)) return set_err(CI_ERR_INVALID_ARG, "decode: max_ctx %u not in 1..2^24", c->max_ctx);
  if (!(c->eps >= 0.0f) || !(c->rope_base > 0.0f)) return set_err(CI_ERR_INVALID_ARG, "decode: eps must be >= 0 and rope_base > 0");
  if ((uint64_t)(c->n_q + 2 * c->n_kv) * c->head_dim > 0xFFFFFFFFull || (uint64_t)c->n_q * c->head_dim > 0xFFFFFFFFull)
    return set_err(CI_ERR_INVALID_ARG, "decode: too many heads");
  return CI_OK;
}

Work work_of(const ci_decode_config_t& c) {
  Work w{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t r = o;
    o = al256(o + bytes);
    return r;
  };
  const size_t B = c.batch, d = c.head_dim;
  w.nchunks = (c.max_ctx + kChunk - 1) / kChunk;
  w.x = take(B * c.hidden * 4);
  w.xn = take(B * c.hidden * 2);
  w.qkv = take(B * (c.n_q + 2 * c.n_kv) * d * 4);
  w.qrot = take(B * c.n_q * d * 4);
  w.part = take(B * c.n_q * w.nchunks * (d + 2) * 4);
  w.attn = take(B * c.n_q * d * 2);
  w.gu = take(B * 2 * (size_t)c.ffn * 4);
  w.h = take(B * c.ffn * 2);
  w.total = o;
  return w;
}

ci_decode_layout_t layout_of(const ci_decode_config_t& c) {
  ci_decode_layout_t L{};
  const uint64_t hid = c.hidden, d = c.head_dim, f = c.ffn;
  uint64_t o = 0;
  auto take = [&](uint64_t elems) {
    const uint64_t r = o;
    o = al64(o + elems);
    return r;
  };
  L.g_attn = take(hid);
  L.w_qkv = take((uint64_t)(c.n_q + 2 * c.n_kv) * d * hid);
  L.w_o = take(hid * c.n_q * d);
  L.g_mlp = take(hid);
  L.w_gu = take(2 * f * hid);
  L.w_down = take(hid * f);
  L.layer_stride = o;
  o = L.layer_stride * c.layers;
  L.g_final = take(hid);
  L.w_lm = take((uint64_t)c.vocab * hid);
  L.weight_elems = o;
  L.cache_elems = (uint64_t)c.layers * c.batch * c.n_kv * c.max_ctx * d;
  const Work w = work_of(c);
  L.workspace_bytes = w.total;
  L.attn_part_bytes = (uint64_t)c.batch * c.n_q * w.nchunks * (d + 2) * 4;
  return L;
}

ci_status_t ensure_decode_state(ci_ctx* ctx, size_t nevents) {
  if (!ctx->dec_pos_host) {
    HIPCHK(hipHostMalloc((void**)&ctx->dec_pos_host, kDecodeMaxBatch * sizeof(int32_t)));
    HIPCHK(hipMalloc((void**)&ctx->dec_pos_dev, 256));
  }
  while (ctx->dec_ev.size() < nevents) {
    hipEvent_t e = nullptr;
    HIPCHK(hipEventCreate(&e));
    ctx->dec_ev.push_back(e);
  }
  return CI_OK;
}

// Validate host positions and queue their copy to the device on `s`.
ci_status_t stage_positions(ci_ctx* ctx, const int32_t* pos, uint32_t batch, uint32_t max_ctx,
                            hipStream_t s, uint32_t* max_pos) {
  if (!pos) return set_err(CI_ERR_INVALID_ARG, "decode: NULL positions");
  uint32_t mp = 0;
  for (uint32_t b = 0; b < batch; ++b) {
    if (pos[b] < 0 || (uint32_t)pos[b] >= max_ctx)
      return set_err(CI_ERR_INVALID_ARG, "decode: position %d of sequence %u not in [0, %u)", pos[b], b, max_ctx);
    mp = std::max(mp, (uint32_t)pos[b]);
  }
  ci_status_t st = ensure_decode_state(ctx, 0);
  if (st != CI_OK) return st;
  memcpy(ctx->dec_pos_host, pos, batch * sizeof(int32_t));
  HIPCHK(hipMemcpyAsync(ctx->dec_pos_dev, ctx->dec_pos_host, batch * sizeof(int32_t),
                        hipMemcpyHostToDevice, s));
  *max_pos = mp;
  return CI_OK;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

ci_status_t check_desc(const ci_decode_desc_t* d) {
  if (!d) return set_err(CI_ERR_INVALID_ARG, "decode: NULL descriptor");
  ci_status_t st = check_cfg(&d->cfg);
  if (st != CI_OK) return st;
  if (!d->weights || !d->k_cache || !d->v_cache || !d->x_in || !d->x_out || !d->work)
    return set_err(CI_ERR_INVALID_ARG, "decode: NULL device pointer");
  if (d->cfg.vocab && !d->logits) return set_err(CI_ERR_INVALID_ARG, "decode: NULL logits with vocab %u", d->cfg.vocab);
  if (!aligned16(d->weights) || !aligned16(d->x_in) || !aligned16(d->x_out) || !aligned16(d->work) ||
      !aligned16(d->k_cache) || !aligned16(d->v_cache))
    return set_err(CI_ERR_INVALID_ARG, "decode: device buffers must be 16-byte aligned");
  return CI_OK;
}

// Order `xs` after the caller's queued work (NULL caller: no ordering).
ci_status_t exec_begin(ci_ctx* ctx, hipStream_t caller, hipStream_t xs) {
  if (caller) {
    HIPCHK(hipEventRecord(ctx->ev[6], caller));
    HIPCHK(hipStreamWaitEvent(xs, ctx->ev[6], 0));
  }
  return CI_OK;
}

ci_status_t exec_end(ci_ctx* ctx, hipStream_t caller, hipStream_t xs) {
  HIPCHK(hipEventRecord(ctx->ev[9], xs));
  if (caller) HIPCHK(hipStreamWaitEvent(caller, ctx->ev[9], 0));
  HIPCHK(hipEventSynchronize(ctx->ev[9]));
  return CI_OK;
}

// One step on exec stream `xs`; blocks until done.
ci_status_t run_decode(ci_ctx* ctx, const ci_decode_desc_t* d, hipStream_t caller, hipStream_t xs,
                       ci_decode_result_t* out) {
  const ci_decode_config_t& c = d->cfg;
  const ci_decode_layout_t L = layout_of(c);
  const Work W = work_of(c);
  const uint32_t nk = c.layers * 10 + (c.vocab ? 2 : 0);
  ci_status_t st = ensure_decode_state(ctx, 2 * (size_t)nk);
  if (st != CI_OK) return st;
  st = exec_begin(ctx, caller, xs);
  if (st != CI_OK) return st;
  uint32_t max_pos = 0;
  st = stage_positions(ctx, d->pos, c.batch, c.max_ctx, xs, &max_pos);
  if (st != CI_OK) return st;
  uint8_t* w8 = (uint8_t*)d->work;
  float* x = (float*)(w8 + W.x);
  uint16_t* xn = (uint16_t*)(w8 + W.xn);
  float* qkv = (float*)(w8 + W.qkv);
  float* qrot = (float*)(w8 + W.qrot);
  float* part = (float*)(w8 + W.part);
  uint16_t* attn = (uint16_t*)(w8 + W.attn);
  float* gu = (float*)(w8 + W.gu);
  uint16_t* h = (uint16_t*)(w8 + W.h);
  const int32_t* pos = ctx->dec_pos_dev;
  const uint32_t B = c.batch, hid = c.hidden, dh = c.head_dim, f = c.ffn;
  const uint32_t qkv_rows = (c.n_q + 2 * c.n_kv) * dh, qd = c.n_q * dh;
  const uint32_t used = max_pos / kChunk + 1;
  const uint64_t cache_layer = (uint64_t)B * c.n_kv * c.max_ctx * dh;
  std::vector<int> kinds;
  kinds.reserve(nk);
  volatile uint64_t* hr = ctx->hres;
  hr[0] = hr[1] = hr[2] = hr[3] = 0;
  HIPCHK(launch_stamp((uint64_t*)&hr[0], xs));
  auto ev = [&](int kind, int which) {
    if (which == 0) kinds.push_back(kind);
    return ctx->dec_ev[2 * (kinds.size() - 1) + which];
  };
#define STEP(kind, call)                                                                       \
  do {                                                                                         \
    hipEvent_t e0_ = ev(kind, 0), e1_ = ev(kind, 1);                                           \
    hipError_t r_ = (call);                                                                    \
    if (r_ != hipSuccess) return set_err(CI_ERR_HIP, "decode %s: %s", #kind, hipGetErrorString(r_)); \
  } while (0)
  const uint16_t* wts = (const uint16_t*)d->weights;
  for (uint32_t l = 0; l < c.layers; ++l) {
    const uint16_t* wl = wts + (uint64_t)l * L.layer_stride;
    uint16_t* kc = (uint16_t*)d->k_cache + l * cache_layer;
    uint16_t* vc = (uint16_t*)d->v_cache + l * cache_layer;
    const float* xres = l == 0 ? d->x_in : x;
    float* xo = l + 1 == c.layers ? d->x_out : x;
    STEP(CI_DK_ATTN_NORM, launch_rmsnorm_bf16(xres, wl + L.g_attn, xn, B, hid, c.eps, xs, e0_, e1_));
    STEP(CI_DK_QKV, launch_gemv_rows(wl + L.w_qkv, xn, nullptr, qkv, qkv_rows, hid, B, xs, e0_, e1_));
    STEP(CI_DK_ROPE, launch_rope_append(qkv, pos, qrot, kc, vc, B, c.n_q, c.n_kv, dh, c.max_ctx,
                                        c.rope_base, xs, e0_, e1_));
    STEP(CI_DK_ATTN, launch_attn_partial(qrot, kc, vc, pos, part, B, c.n_q, c.n_kv, dh, c.max_ctx,
                                         W.nchunks, used, xs, e0_, e1_));
    STEP(CI_DK_ATTN_COMBINE, launch_attn_combine(part, pos, attn, B, c.n_q, dh, W.nchunks, xs, e0_, e1_));
    STEP(CI_DK_OPROJ, launch_gemv_rows(wl + L.w_o, attn, xres, x, hid, qd, B, xs, e0_, e1_));
    STEP(CI_DK_MLP_NORM, launch_rmsnorm_bf16(x, wl + L.g_mlp, xn, B, hid, c.eps, xs, e0_, e1_));
    STEP(CI_DK_GATE_UP, launch_gemv_rows(wl + L.w_gu, xn, nullptr, gu, 2 * f, hid, B, xs, e0_, e1_));
    STEP(CI_DK_SILU, launch_silu_mul(gu, h, f, B, xs, e0_, e1_));
    STEP(CI_DK_DOWN, launch_gemv_rows(wl + L.w_down, h, x, xo, hid, f, B, xs, e0_, e1_));
  }
  if (c.vocab) {
    STEP(CI_DK_FINAL_NORM, launch_rmsnorm_bf16(d->x_out, wts + L.g_final, xn, B, hid, c.eps, xs, e0_, e1_));
    STEP(CI_DK_LM_HEAD, launch_gemv_rows(wts + L.w_lm, xn, nullptr, d->logits, c.vocab, hid, B, xs, e0_, e1_));
  }
#undef STEP
  HIPCHK(launch_stamp((uint64_t*)&hr[1], xs));
  const float* res = c.vocab ? d->logits : d->x_out;
  const uint64_t len = (uint64_t)B * (c.vocab ? c.vocab : hid);
  HIPCHK(launch_checksum_f32(res, len, ctx->part_bits, ctx->part_sum, ctx->nparts, (uint64_t*)&hr[2],
                             (double*)&hr[3], xs));
  st = exec_end(ctx, caller, xs);
  if (st != CI_OK) return st;
  memset(out, 0, sizeof(*out));
  for (size_t i = 0; i < kinds.size(); ++i) {
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, ctx->dec_ev[2 * i], ctx->dec_ev[2 * i + 1]));
    out->kernel_ns[kinds[i]] += (double)ms * 1e6;
  }
  float ms = 0.0f;
  HIPCHK(hipEventElapsedTime(&ms, ctx->dec_ev[0], ctx->dec_ev[2 * kinds.size() - 1]));
  out->step_ns = (double)ms * 1e6;
  out->t_begin = hr[0];
  out->t_end = hr[1];
  out->checksum_bits = hr[2];
  uint64_t sb = hr[3];
  memcpy(&out->sum_f64, &sb, sizeof(double));
  return CI_OK;
}

}  // namespace

extern "C" ci_status_t decode_layout(const ci_decode_config_t* cfg, ci_decode_layout_t* out) {
  if (!out) return set_err(CI_ERR_INVALID_ARG, "decode_layout: NULL output");
  ci_status_t st = check_cfg(cfg);
  if (st != CI_OK) return st;
  *out = layout_of(*cfg);
  return CI_OK;
}

extern "C" ci_status_t decode_step(ci_ctx_t* ctx, const ci_decode_desc_t* d, void* stream,
                                   ci_decode_result_t* out) {
  if (!ctx || !out) return set_err(CI_ERR_INVALID_ARG, "decode_step: NULL argument");
  ci_status_t st = check_desc(d);
  if (st != CI_OK) return st;
  HIPCHK(hipSetDevice(ctx->device));
  return run_decode(ctx, d, (hipStream_t)stream, ctx->vstream, out);
}

extern "C" ci_status_t measure_decode(ci_ctx_t* ctx, const ci_decode_desc_t* d,
                                      const ci_resource_t* rs, const ci_stressor_opts_t* sopts,
                                      int nr, const float* xs, int nx, const ci_measure_opts_t* o,
                                      void* ws, size_t ws_bytes, void* stream,
                                      ci_decode_cell_t* cells) {
  if (!ctx || !rs || !xs || !cells || nr <= 0 || nx <= 0)
    return set_err(CI_ERR_INVALID_ARG, "measure_decode: bad argument");
  ci_status_t st = check_desc(d);
  if (st != CI_OK) return st;
  ci_measure_opts_t mo{20, 3, CI_PLACE_SHARED, 2000};
  if (o) {
    mo = *o;
    if (!mo.reps) mo.reps = 20;
    if (!mo.deadline_ms) mo.deadline_ms = 2000;
  }
  for (int j = 0; j < nx; ++j)
    if (!(xs[j] >= 0.0f && xs[j] <= 1.0f))
      return set_err(CI_ERR_INVALID_ARG, "measure_decode: intensity %g", xs[j]);
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t caller = (hipStream_t)stream;
  for (int i = 0; i < nr; ++i) {
    for (int j = 0; j < nx; ++j) {
      ci_decode_cell_t& cell = cells[i * nx + j];
      memset(&cell, 0, sizeof(cell));
      cell.resource = rs[i];
      cell.intensity = xs[j];
      cell.duty = sopts ? (sopts[i].duty ? sopts[i].duty : 100) : 100;
      const int k = cus_for(ctx, xs[j]);
      cell.ncu = k;
      hipStream_t vs = ctx->vstream;
      if (mo.placement == CI_PLACE_DISJOINT) {
        if (k >= ctx->info.num_cus) {
          cell.step_alone_p50 = cell.step_col_p50 = NAN;
          continue;
        }
        uint32_t mask[8];
        mask_for(ctx, k, 1, mask);
        vs = masked_stream(ctx, mask);
        if (!vs) return set_err(CI_ERR_HIP, "hipExtStreamCreateWithCUMask failed");
      }
      ci_stressor_opts_t so{};
      if (sopts) so = sopts[i];
      so.passes = 0;
      so.deadline_ms = mo.deadline_ms;
      ci_decode_result_t r;
      for (uint32_t w = 0; w < mo.warmups; ++w) {
        st = run_decode(ctx, d, caller, vs, &r);
        if (st != CI_OK) return st;
      }
      std::vector<double> ta, tc;
      std::vector<double> ka[CI_DK_COUNT], kcol[CI_DK_COUNT];
      double ach = 0.0, pct = 0.0;
      int covered = 1, equal = 1, timed = 0, nrep = 0;
      for (uint32_t rep = 0; rep < mo.reps; ++rep) {
        ci_decode_result_t ra, rc;
        st = run_decode(ctx, d, caller, vs, &ra);
        if (st != CI_OK) return st;
        ci_stressor_t* h = nullptr;
        st = stressor_launch(ctx, rs[i], xs[j], caller, &so, ws, ws_bytes, &h);
        if (st != CI_OK) return st;
        ci_status_t vst = run_decode(ctx, d, caller, vs, &rc);
        ci_stressor_report_t sr;
        const bool noop = h->noop;
        st = stressor_stop(h, &sr);
        if (vst != CI_OK) return vst;
        if (st == CI_ERR_TIMEOUT) {
          timed = 1;
        } else if (st != CI_OK) {
          return st;
        }
        if (!noop && rs[i] != CI_RES_DISPATCH) {
          if (!(sr.t_last_start <= rc.t_begin && sr.t_first_end >= rc.t_end) || sr.wg_reported != sr.grid)
            covered = 0;
        }
        if (rc.checksum_bits != ra.checksum_bits) equal = 0;
        ta.push_back(ra.step_ns);
        tc.push_back(rc.step_ns);
        for (int q = 0; q < CI_DK_COUNT; ++q) {
          ka[q].push_back(ra.kernel_ns[q]);
          kcol[q].push_back(rc.kernel_ns[q]);
        }
        ach += sr.achieved;
        pct += sr.pct_of_peak;
        ++nrep;
      }
      cell.reps = nrep;
      cell.step_alone_p50 = quantile(ta, 0.5);
      cell.step_alone_p90 = quantile(ta, 0.9);
      cell.step_col_p50 = quantile(tc, 0.5);
      cell.step_col_p90 = quantile(tc, 0.9);
      for (int q = 0; q < CI_DK_COUNT; ++q) {
        cell.kernel_alone_ns[q] = median(ka[q]);
        cell.kernel_col_ns[q] = median(kcol[q]);
      }
      cell.stressor_achieved = nrep ? ach / nrep : 0.0;
      cell.stressor_pct_peak = nrep ? pct / nrep : 0.0;
      cell.window_covered = covered;
      cell.output_equal = equal;
      cell.timed_out = timed;
    }
  }
  return CI_OK;
}

// ------------------------------------------------------- kernels one by one
extern "C" ci_status_t ci_rmsnorm_bf16(ci_ctx_t* ctx, const float* x, const uint16_t* g, uint32_t rows,
                                       uint32_t n, float eps, uint16_t* y, void* stream) {
  if (!ctx || !x || !g || !y) return set_err(CI_ERR_INVALID_ARG, "ci_rmsnorm_bf16: NULL argument");
  if (rows == 0 || n == 0 || n % 4) return set_err(CI_ERR_INVALID_ARG, "ci_rmsnorm_bf16: n must be a positive multiple of 4");
  if (((uintptr_t)x & 15) || ((uintptr_t)g & 7) || ((uintptr_t)y & 7))
    return set_err(CI_ERR_INVALID_ARG, "ci_rmsnorm_bf16: misaligned buffer");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t caller = (hipStream_t)stream, xs = ctx->vstream;
  ci_status_t st = exec_begin(ctx, caller, xs);
  if (st != CI_OK) return st;
  HIPCHK(launch_rmsnorm_bf16(x, g, y, rows, n, eps, xs, nullptr, nullptr));
  return exec_end(ctx, caller, xs);
}

extern "C" ci_status_t ci_gemv_bf16_rows(ci_ctx_t* ctx, const uint16_t* w, const uint16_t* v,
                                         const float* res, float* out, uint32_t rows, uint32_t k,
                                         uint32_t batch, void* stream) {
  if (!ctx || !w || !v || !out) return set_err(CI_ERR_INVALID_ARG, "ci_gemv_bf16_rows: NULL argument");
  if (rows == 0 || k == 0 || k % 8) return set_err(CI_ERR_INVALID_ARG, "ci_gemv_bf16_rows: k must be a positive multiple of 8");
  if (batch == 0 || batch > kDecodeMaxBatch) return set_err(CI_ERR_INVALID_ARG, "ci_gemv_bf16_rows: batch %u not in 1..8", batch);
  if (!aligned16(w) || !aligned16(v)) return set_err(CI_ERR_INVALID_ARG, "ci_gemv_bf16_rows: w and v must be 16-byte aligned");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t caller = (hipStream_t)stream, xs = ctx->vstream;
  ci_status_t st = exec_begin(ctx, caller, xs);
  if (st != CI_OK) return st;
  HIPCHK(launch_gemv_rows(w, v, res, out, rows, k, batch, xs, nullptr, nullptr));
  return exec_end(ctx, caller, xs);
}

extern "C" ci_status_t ci_rope_append(ci_ctx_t* ctx, const float* qkv, const int32_t* pos, uint32_t batch,
                                      uint32_t n_q, uint32_t n_kv, uint32_t head_dim, uint32_t max_ctx,
                                      float rope_base, float* q_out, uint16_t* k_cache,
                                      uint16_t* v_cache, void* stream) {
  if (!ctx || !qkv || !q_out || !k_cache || !v_cache) return set_err(CI_ERR_INVALID_ARG, "ci_rope_append: NULL argument");
  ci_decode_config_t c{8, n_q, n_kv, head_dim, 8, 0, 1, batch, max_ctx, 0.0f, rope_base};
  ci_status_t st = check_cfg(&c);
  if (st != CI_OK) return st;
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t caller = (hipStream_t)stream, xs = ctx->vstream;
  st = exec_begin(ctx, caller, xs);
  if (st != CI_OK) return st;
  uint32_t mp = 0;
  st = stage_positions(ctx, pos, batch, max_ctx, xs, &mp);
  if (st != CI_OK) return st;
  HIPCHK(launch_rope_append(qkv, ctx->dec_pos_dev, q_out, k_cache, v_cache, batch, n_q, n_kv, head_dim,
                            max_ctx, rope_base, xs, nullptr, nullptr));
  return exec_end(ctx, caller, xs);
}

extern "C" ci_status_t ci_attention_decode(ci_ctx_t* ctx, const float* q, const uint16_t* k_cache,
                                           const uint16_t* v_cache, const int32_t* pos, uint32_t batch,
                                           uint32_t n_q, uint32_t n_kv, uint32_t head_dim,
                                           uint32_t max_ctx, void* part, size_t part_bytes,
                                           uint16_t* out, void* stream) {
  if (!ctx || !q || !k_cache || !v_cache || !part || !out)
    return set_err(CI_ERR_INVALID_ARG, "ci_attention_decode: NULL argument");
  ci_decode_config_t c{8, n_q, n_kv, head_dim, 8, 0, 1, batch, max_ctx, 0.0f, 1.0f};
  ci_status_t st = check_cfg(&c);
  if (st != CI_OK) return st;
  const ci_decode_layout_t L = layout_of(c);
  if (part_bytes < L.attn_part_bytes)
    return set_err(CI_ERR_INVALID_ARG, "ci_attention_decode: part %zu bytes < %llu needed", part_bytes,
                   (unsigned long long)L.attn_part_bytes);
  if (!aligned16(k_cache) || !aligned16(v_cache)) return set_err(CI_ERR_INVALID_ARG, "ci_attention_decode: misaligned cache");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t caller = (hipStream_t)stream, xs = ctx->vstream;
  st = exec_begin(ctx, caller, xs);
  if (st != CI_OK) return st;
  uint32_t mp = 0;
  st = stage_positions(ctx, pos, batch, max_ctx, xs, &mp);
  if (st != CI_OK) return st;
  const uint32_t nchunks = (max_ctx + kChunk - 1) / kChunk;
  HIPCHK(launch_attn_partial(q, k_cache, v_cache, ctx->dec_pos_dev, (float*)part, batch, n_q, n_kv, head_dim,
                             max_ctx, nchunks, mp / kChunk + 1, xs, nullptr, nullptr));
  HIPCHK(launch_attn_combine((const float*)part, ctx->dec_pos_dev, out, batch, n_q, head_dim, nchunks, xs,
                             nullptr, nullptr));
  return exec_end(ctx, caller, xs);
}

extern "C" ci_status_t ci_silu_mul_bf16(ci_ctx_t* ctx, const float* gu, uint32_t batch, uint32_t ffn,
                                        uint16_t* h, void* stream) {
  if (!ctx || !gu || !h) return set_err(CI_ERR_INVALID_ARG, "ci_silu_mul_bf16: NULL argument");
  if (batch == 0 || ffn == 0) return set_err(CI_ERR_INVALID_ARG, "ci_silu_mul_bf16: empty shape");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t caller = (hipStream_t)stream, xs = ctx->vstream;
  ci_status_t st = exec_begin(ctx, caller, xs);
  if (st != CI_OK) return st;
  HIPCHK(launch_silu_mul(gu, h, ffn, batch, xs, nullptr, nullptr));
  return exec_end(ctx, caller, xs);
}
