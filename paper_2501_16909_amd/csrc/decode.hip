// Host runtime of the synthetic decode step: config validation and layouts,
// the step itself (one timed launch per kernel), the kernels one at a time,
// and the step's sensitivity measurement beside a stressor.
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "runtime.h"

using namespace ci;

namespace {

constexpr uint32_t kChunk = 64;   // attention positions per work-group

uint64_t al64(uint64_t x) { return (x + 63) & ~63ull; }
size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Work {
  size_t x, qrot, part, attn, h, total;
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
  w.qrot = take(B * c.n_q * d * 4);
  w.part = take(B * c.n_q * w.nchunks * (d + 2) * 4);
  w.attn = take(B * c.n_q * d * 2);
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
  if (d->flags & ~(CI_DECODE_KERNEL_TIMES | CI_DECODE_GRAPH) ||
      (d->flags & CI_DECODE_KERNEL_TIMES && d->flags & CI_DECODE_GRAPH))
    return set_err(CI_ERR_INVALID_ARG, "decode: flags 0x%x", d->flags);
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

// Queue the step's kernels on `xs`.  ev(kind) gives the event pair of the
// next launch (both null for untimed launches).
template <class EvFn>
ci_status_t enqueue_step(const ci_decode_desc_t* d, const int32_t* pos, uint32_t used, hipStream_t xs,
                         EvFn ev) {
  const ci_decode_config_t& c = d->cfg;
  const ci_decode_layout_t L = layout_of(c);
  const Work W = work_of(c);
  uint8_t* w8 = (uint8_t*)d->work;
  float* x = (float*)(w8 + W.x);
  float* qrot = (float*)(w8 + W.qrot);
  float* part = (float*)(w8 + W.part);
  uint16_t* attn = (uint16_t*)(w8 + W.attn);
  uint16_t* h = (uint16_t*)(w8 + W.h);
  const uint32_t B = c.batch, hid = c.hidden, dh = c.head_dim, f = c.ffn;
  const uint64_t cache_layer = (uint64_t)B * c.n_kv * c.max_ctx * dh;
  const uint16_t* wts = (const uint16_t*)d->weights;
#define STEP(kind, call)                                                                       \
  do {                                                                                         \
    hipEvent_t e0_, e1_;                                                                       \
    ev(kind, &e0_, &e1_);                                                                      \
    hipError_t r_ = (call);                                                                    \
    if (r_ != hipSuccess) return set_err(CI_ERR_HIP, "decode %s: %s", #kind, hipGetErrorString(r_)); \
  } while (0)
  for (uint32_t l = 0; l < c.layers; ++l) {
    const uint16_t* wl = wts + (uint64_t)l * L.layer_stride;
    const float* xres = l == 0 ? d->x_in : x;
    float* xo = l + 1 == c.layers ? d->x_out : x;
    GemvArgs q{};
    q.w = wl + L.w_qkv;
    q.x = xres;
    q.g = wl + L.g_attn;
    q.eps = c.eps;
    q.pos = pos;
    q.q_out = qrot;
    q.kc = (uint16_t*)d->k_cache + l * cache_layer;
    q.vc = (uint16_t*)d->v_cache + l * cache_layer;
    q.rows = (c.n_q + 2 * c.n_kv) * dh;
    q.k = hid;
    q.batch = B;
    q.nq = c.n_q;
    q.nkv = c.n_kv;
    q.d = dh;
    q.max_ctx = c.max_ctx;
    q.base = c.rope_base;
    STEP(CI_DK_QKV, launch_gemv_fused(q, 1, kEpiRope, xs, e0_, e1_));
    STEP(CI_DK_ATTN, launch_attn_partial(qrot, q.kc, q.vc, pos, part, B, c.n_q, c.n_kv, dh, c.max_ctx,
                                         W.nchunks, used, xs, e0_, e1_));
    STEP(CI_DK_ATTN_COMBINE, launch_attn_combine(part, pos, attn, B, c.n_q, dh, W.nchunks, xs, e0_, e1_));
    GemvArgs o{};
    o.w = wl + L.w_o;
    o.v = attn;
    o.res = xres;
    o.out = x;
    o.rows = hid;
    o.k = c.n_q * dh;
    o.batch = B;
    STEP(CI_DK_OPROJ, launch_gemv_fused(o, 0, kEpiPlain, xs, e0_, e1_));
    GemvArgs g{};
    g.w = wl + L.w_gu;
    g.x = x;
    g.g = wl + L.g_mlp;
    g.eps = c.eps;
    g.h = h;
    g.rows = 2 * f;
    g.k = hid;
    g.batch = B;
    STEP(CI_DK_GATE_UP, launch_gemv_fused(g, 1, kEpiSilu, xs, e0_, e1_));
    GemvArgs dn{};
    dn.w = wl + L.w_down;
    dn.v = h;
    dn.res = x;
    dn.out = xo;
    dn.rows = hid;
    dn.k = f;
    dn.batch = B;
    STEP(CI_DK_DOWN, launch_gemv_fused(dn, 0, kEpiPlain, xs, e0_, e1_));
  }
  if (c.vocab) {
    GemvArgs lm{};
    lm.w = wts + L.w_lm;
    lm.x = d->x_out;
    lm.g = wts + L.g_final;
    lm.eps = c.eps;
    lm.out = d->logits;
    lm.rows = c.vocab;
    lm.k = hid;
    lm.batch = B;
    STEP(CI_DK_LM_HEAD, launch_gemv_fused(lm, 1, kEpiPlain, xs, e0_, e1_));
  }
#undef STEP
  return CI_OK;
}

uint32_t launches_of(const ci_decode_config_t& c) { return c.layers * 6 + (c.vocab ? 1 : 0); }

// Graph of the step's launches for this descriptor (everything but the
// host positions) and context bucket, captured on first use.
ci_status_t step_graph(ci_ctx* ctx, const ci_decode_desc_t* d, uint32_t used, hipStream_t xs,
                       hipGraphExec_t* out) {
  std::string key((const char*)d, offsetof(ci_decode_desc_t, pos));
  key.append((const char*)&d->x_in, offsetof(ci_decode_desc_t, flags) - offsetof(ci_decode_desc_t, x_in));
  key.append((const char*)&used, sizeof(used));
  key.append((const char*)&xs, sizeof(xs));
  auto it = ctx->dec_graphs.find(key);
  if (it != ctx->dec_graphs.end()) {
    *out = it->second;
    return CI_OK;
  }
  if (ctx->dec_graphs.size() >= kDecodeMaxGraphs) {
    (void)hipGraphExecDestroy(ctx->dec_graphs.begin()->second);
    ctx->dec_graphs.erase(ctx->dec_graphs.begin());
  }
  HIPCHK(hipStreamBeginCapture(xs, hipStreamCaptureModeRelaxed));
  ci_status_t st = enqueue_step(d, ctx->dec_pos_dev, used, xs, [](int, hipEvent_t* a, hipEvent_t* b) {
    *a = *b = nullptr;
  });
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(xs, &g);
  if (st != CI_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (ec != hipSuccess) return set_err(CI_ERR_HIP, "decode graph capture: %s", hipGetErrorString(ec));
  hipGraphExec_t ex = nullptr;
  const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) return set_err(CI_ERR_HIP, "decode graph instantiate: %s", hipGetErrorString(ei));
  ctx->dec_graphs.emplace(key, ex);
  *out = ex;
  return CI_OK;
}

ci_status_t run_decode(ci_ctx* ctx, const ci_decode_desc_t* d, hipStream_t caller, hipStream_t xs,
                       ci_decode_result_t* out);

struct DecodeRun {
  ci_ctx* ctx;
  const ci_decode_desc_t* d;
  hipStream_t caller;
  static ci_status_t call(void* p, hipStream_t vs, double* ns) {
    DecodeRun* v = static_cast<DecodeRun*>(p);
    ci_decode_result_t r;
    const ci_status_t st = run_decode(v->ctx, v->d, v->caller, vs, &r);
    *ns = r.step_ns;
    return st;
  }
};

// One step on exec stream `xs`; blocks until done.
ci_status_t run_decode(ci_ctx* ctx, const ci_decode_desc_t* d, hipStream_t caller, hipStream_t xs,
                       ci_decode_result_t* out) {
  const ci_decode_config_t& c = d->cfg;
  const uint32_t nk = launches_of(c);
  const bool timed = d->flags & CI_DECODE_KERNEL_TIMES;
  ci_status_t st = ensure_decode_state(ctx, timed ? 2 * (size_t)nk : 0);
  if (st != CI_OK) return st;
  if (!d->pos) return set_err(CI_ERR_INVALID_ARG, "decode: NULL positions");
  uint32_t max_pos = 0;
  for (uint32_t b = 0; b < c.batch; ++b) {   // before any capture or launch
    if (d->pos[b] < 0 || (uint32_t)d->pos[b] >= c.max_ctx)
      return set_err(CI_ERR_INVALID_ARG, "decode: position %d of sequence %u not in [0, %u)", d->pos[b], b,
                     c.max_ctx);
    max_pos = std::max(max_pos, (uint32_t)d->pos[b]);
  }
  const uint32_t used = max_pos / kChunk + 1;
  hipGraphExec_t graph = nullptr;
  if (d->flags & CI_DECODE_GRAPH) {
    st = step_graph(ctx, d, used, xs, &graph);
    if (st != CI_OK) return st;
  }
  st = exec_begin(ctx, caller, xs);
  if (st != CI_OK) return st;
  st = stage_positions(ctx, d->pos, c.batch, c.max_ctx, xs, &max_pos);
  if (st != CI_OK) return st;
  volatile uint64_t* hr = ctx->hres;
  hr[0] = hr[1] = hr[2] = hr[3] = 0;
  HIPCHK(launch_stamp((uint64_t*)&hr[0], xs));
  std::vector<int> kinds;
  if (graph) {
    HIPCHK(hipEventRecord(ctx->ev[7], xs));
    HIPCHK(hipGraphLaunch(graph, xs));
    HIPCHK(hipEventRecord(ctx->ev[8], xs));
  } else if (timed) {
    kinds.reserve(nk);
    st = enqueue_step(d, ctx->dec_pos_dev, used, xs, [&](int kind, hipEvent_t* a, hipEvent_t* b) {
      kinds.push_back(kind);
      *a = ctx->dec_ev[2 * (kinds.size() - 1)];
      *b = ctx->dec_ev[2 * (kinds.size() - 1) + 1];
    });
    if (st != CI_OK) return st;
  } else {
    HIPCHK(hipEventRecord(ctx->ev[7], xs));
    st = enqueue_step(d, ctx->dec_pos_dev, used, xs, [](int, hipEvent_t* a, hipEvent_t* b) {
      *a = *b = nullptr;
    });
    if (st != CI_OK) return st;
    HIPCHK(hipEventRecord(ctx->ev[8], xs));
  }
  HIPCHK(launch_stamp((uint64_t*)&hr[1], xs));
  const float* res = c.vocab ? d->logits : d->x_out;
  const uint64_t len = (uint64_t)c.batch * (c.vocab ? c.vocab : c.hidden);
  HIPCHK(launch_checksum_f32(res, len, ctx->part_bits, ctx->part_sum, ctx->nparts, (uint64_t*)&hr[2],
                             (double*)&hr[3], xs));
  st = exec_end(ctx, caller, xs);
  if (st != CI_OK) return st;
  memset(out, 0, sizeof(*out));
  float ms = 0.0f;
  if (timed) {
    for (size_t i = 0; i < kinds.size(); ++i) {
      HIPCHK(hipEventElapsedTime(&ms, ctx->dec_ev[2 * i], ctx->dec_ev[2 * i + 1]));
      out->kernel_ns[kinds[i]] += (double)ms * 1e6;
    }
    HIPCHK(hipEventElapsedTime(&ms, ctx->dec_ev[0], ctx->dec_ev[2 * kinds.size() - 1]));
  } else {
    HIPCHK(hipEventElapsedTime(&ms, ctx->ev[7], ctx->ev[8]));
  }
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
  ci_measure_opts_t mo{20, 3, CI_PLACE_SHARED, 2000, 0};
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
  ctx->queue_checked.clear();  // queue pairs are checked per victim
  ctx->queue_qualified.clear();
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
      HeldStream hold(ctx, &vs);  // the cache never evicts the victim's stream
      uint32_t vmask[8];
      const bool masked = mo.placement == CI_PLACE_DISJOINT && k > 0;  // k == 0: whole GPU, unmasked
      if (masked) {
        if (k >= ctx->info.num_cus) {
          cell.step_alone_p50 = cell.step_col_p50 = NAN;
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
      ci_decode_result_t r;
      DecodeRun dr{ctx, d, caller};
      if (!(mo.flags & CI_MEASURE_NO_QUEUE_CHECK)) {
        st = check_queue_pair(ctx, rs[i], sopts ? &sopts[i] : nullptr, xs[j], caller, &vs,
                              masked ? vmask : nullptr, ws, ws_bytes, &DecodeRun::call, &dr,
                              &cell.queue_unresolved);
        if (st != CI_OK) return st;
      }
      for (uint32_t w = 0; w < mo.warmups; ++w) {
        st = run_decode(ctx, d, caller, vs, &r);
        if (st != CI_OK) return st;
      }
      std::vector<double> ta, tc;
      std::vector<double> ka[CI_DK_COUNT], kcol[CI_DK_COUNT];
      double ach = 0.0, pct = 0.0;
      int covered = 1, equal = 1, timed = 0, nrep = 0;
      for (uint32_t rep = 0; rep < mo.reps; ++rep) {
        // counterbalanced order, as in measure_sensitivity
        const bool col_first = rep & 1u;
        ci_decode_result_t ra, rc;
        if (!col_first) {
          st = run_decode(ctx, d, caller, vs, &ra);
          if (st != CI_OK) return st;
        }
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
        if (col_first) {
          st = run_decode(ctx, d, caller, vs, &ra);
          if (st != CI_OK) return st;
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
  GemvArgs a{};
  a.w = w;
  a.v = v;
  a.res = res;
  a.out = out;
  a.rows = rows;
  a.k = k;
  a.batch = batch;
  HIPCHK(launch_gemv_fused(a, 0, kEpiPlain, xs, nullptr, nullptr));
  return exec_end(ctx, caller, xs);
}

extern "C" ci_status_t ci_fused_gemv(ci_ctx_t* ctx, const ci_gemv_args_t* in, void* stream) {
  if (!ctx || !in || !in->w) return set_err(CI_ERR_INVALID_ARG, "ci_fused_gemv: NULL argument");
  const ci_gemv_args_t& a = *in;
  if (a.rows == 0 || a.k == 0 || a.k % 8) return set_err(CI_ERR_INVALID_ARG, "ci_fused_gemv: k must be a positive multiple of 8");
  if (a.batch == 0 || a.batch > kDecodeMaxBatch) return set_err(CI_ERR_INVALID_ARG, "ci_fused_gemv: batch %u not in 1..8", a.batch);
  if (!aligned16(a.w) || (a.v && !aligned16(a.v)) || (!a.v && (!a.x || !a.g || !aligned16(a.x) || !aligned16(a.g))))
    return set_err(CI_ERR_INVALID_ARG, "ci_fused_gemv: input missing or not 16-byte aligned");
  GemvArgs g{};
  g.w = (const uint16_t*)a.w;
  g.v = (const uint16_t*)a.v;
  g.x = a.x;
  g.g = (const uint16_t*)a.g;
  g.eps = a.eps;
  g.rows = a.rows;
  g.k = a.k;
  g.batch = a.batch;
  if (a.epilogue == CI_GEMV_PLAIN) {
    if (!a.out) return set_err(CI_ERR_INVALID_ARG, "ci_fused_gemv: NULL out");
    g.res = a.res;
    g.out = a.out;
  } else if (a.epilogue == CI_GEMV_SILU) {
    if (!a.h || a.rows % 2) return set_err(CI_ERR_INVALID_ARG, "ci_fused_gemv: SILU needs h and an even row count");
    g.h = (uint16_t*)a.h;
  } else if (a.epilogue == CI_GEMV_ROPE) {
    ci_decode_config_t c{8, a.n_q, a.n_kv, a.head_dim, 8, 0, 1, a.batch, a.max_ctx, 0.0f, a.rope_base};
    ci_status_t st = check_cfg(&c);
    if (st != CI_OK) return st;
    if ((uint64_t)(a.n_q + 2 * a.n_kv) * a.head_dim != a.rows)
      return set_err(CI_ERR_INVALID_ARG, "ci_fused_gemv: ROPE rows %u != (n_q + 2 n_kv) * head_dim", a.rows);
    if (!a.q_out || !a.k_cache || !a.v_cache) return set_err(CI_ERR_INVALID_ARG, "ci_fused_gemv: NULL ROPE output");
    g.q_out = a.q_out;
    g.kc = (uint16_t*)a.k_cache;
    g.vc = (uint16_t*)a.v_cache;
    g.nq = a.n_q;
    g.nkv = a.n_kv;
    g.d = a.head_dim;
    g.max_ctx = a.max_ctx;
    g.base = a.rope_base;
  } else {
    return set_err(CI_ERR_INVALID_ARG, "ci_fused_gemv: epilogue %d", a.epilogue);
  }
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t caller = (hipStream_t)stream, xs = ctx->vstream;
  ci_status_t st = exec_begin(ctx, caller, xs);
  if (st != CI_OK) return st;
  if (a.epilogue == CI_GEMV_ROPE) {
    uint32_t mp = 0;
    st = stage_positions(ctx, a.pos, a.batch, a.max_ctx, xs, &mp);
    if (st != CI_OK) return st;
    g.pos = ctx->dec_pos_dev;
  }
  HIPCHK(launch_gemv_fused(g, a.v ? 0 : 1, a.epilogue, xs, nullptr, nullptr));
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

// ------------------------------------------------ no-allocation attention
// ci_attention_decode_noalloc works in this array instead of a caller's
// workspace and the context's lazily allocated position buffer: the first
// 256 bytes hold the positions, the rest the partial results.  Each device
// holds its own copy for the life of the process.  Host code never passes
// the array's name to a kernel (on the host it is only a stand-in for the
// symbol): it uses the address hipGetSymbolAddress gives per device.
namespace {
constexpr size_t kScratchPosBytes = 256;
constexpr size_t kScratchBytes = kScratchPosBytes + CI_NOALLOC_PART_BYTES;
static_assert(kDecodeMaxBatch * sizeof(int32_t) <= kScratchPosBytes, "positions must fit the header");

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kScratchMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchMaxDevices];

struct PosArg {
  int32_t v[kDecodeMaxBatch];
};

// Positions reach the device as a kernel argument (no staging buffer).
__global__ void __launch_bounds__(64) store_positions_kernel(PosArg p, uint32_t batch, int32_t* dst) {
  if (threadIdx.x < batch) dst[threadIdx.x] = p.v[threadIdx.x];
}
}  // namespace

ci_status_t ci::static_scratch_init(int device) {
  if (device < 0 || device >= kScratchMaxDevices)
    return set_err(CI_ERR_UNSUPPORTED, "static scratch: device %d beyond %d", device, kScratchMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return CI_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return set_err(CI_ERR_HIP, "static scratch: hipGetSymbolAddress on device %d: %s", device,
                   hipGetErrorString(e));
  if ((uintptr_t)ptr & 255)
    return set_err(CI_ERR_HIP, "static scratch: device %d address %p not 256-byte aligned", device, ptr);
  g_scratch_ptr[device] = ptr;
  return CI_OK;
}

extern "C" ci_status_t ci_attention_decode_noalloc(ci_ctx_t* ctx, const float* q, const uint16_t* k_cache,
                                                   const uint16_t* v_cache, const int32_t* pos,
                                                   uint32_t batch, uint32_t n_q, uint32_t n_kv,
                                                   uint32_t head_dim, uint32_t max_ctx, uint16_t* out,
                                                   void* stream) {
  if (!ctx || !q || !k_cache || !v_cache || !pos || !out)
    return set_err(CI_ERR_INVALID_ARG, "ci_attention_decode_noalloc: NULL argument");
  ci_decode_config_t c{8, n_q, n_kv, head_dim, 8, 0, 1, batch, max_ctx, 0.0f, 1.0f};
  ci_status_t st = check_cfg(&c);
  if (st != CI_OK) return st;
  const ci_decode_layout_t L = layout_of(c);
  if (L.attn_part_bytes > CI_NOALLOC_PART_BYTES)
    return set_err(CI_ERR_INVALID_ARG,
                   "ci_attention_decode_noalloc: %llu bytes of partial results exceed the static scratch "
                   "limit of %llu (batch x n_q x ceil(max_ctx / 64) x (head_dim + 2) x 4)",
                   (unsigned long long)L.attn_part_bytes, (unsigned long long)CI_NOALLOC_PART_BYTES);
  if (!aligned16(k_cache) || !aligned16(v_cache))
    return set_err(CI_ERR_INVALID_ARG, "ci_attention_decode_noalloc: misaligned cache");
  PosArg pa{};
  uint32_t mp = 0;
  for (uint32_t b = 0; b < batch; ++b) {
    if (pos[b] < 0 || (uint32_t)pos[b] >= max_ctx)
      return set_err(CI_ERR_INVALID_ARG, "ci_attention_decode_noalloc: position %d of sequence %u not in [0, %u)",
                     pos[b], b, max_ctx);
    pa.v[b] = pos[b];
    mp = std::max(mp, (uint32_t)pos[b]);
  }
  void* base = (ctx->device >= 0 && ctx->device < kScratchMaxDevices) ? g_scratch_ptr[ctx->device] : nullptr;
  if (!base) return set_err(CI_ERR_UNSUPPORTED, "ci_attention_decode_noalloc: static scratch not set up");
  int32_t* dpos = (int32_t*)base;
  float* part = (float*)((uint8_t*)base + kScratchPosBytes);
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t caller = (hipStream_t)stream, xs = ctx->vstream;
  st = exec_begin(ctx, caller, xs);
  if (st != CI_OK) return st;
  // every partial entry the combine reads is written by the partial kernel,
  // and the positions are rewritten here: nothing needs clearing
  HIPCHK(xlaunch(store_positions_kernel, dim3(1), dim3(64), 0, xs, nullptr, nullptr, pa, batch, dpos));
  const uint32_t nchunks = (max_ctx + kChunk - 1) / kChunk;
  HIPCHK(launch_attn_partial(q, k_cache, v_cache, dpos, part, batch, n_q, n_kv, head_dim, max_ctx, nchunks,
                             mp / kChunk + 1, xs, nullptr, nullptr));
  HIPCHK(launch_attn_combine(part, dpos, out, batch, n_q, head_dim, nchunks, xs, nullptr, nullptr));
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
