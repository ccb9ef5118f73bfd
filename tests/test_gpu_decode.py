"""GPU parity of the synthetic decode step (the stand-in for the paper's LLM
decode victims) against the FP64 oracle: each kernel alone on seeded
inputs, the whole step on a small model and on one full-width Llama-3.1-8B
layer, and the step's sensitivity measurement beside a stressor.

BF16 outputs: the device rounds its FP32 value, the oracle its FP64 value,
so a code may differ where the two sit on opposite sides of a rounding
boundary.  A code is accepted when it is the rounding of some value within
the kernel's FP32 error bound of the exact result (rounding is monotone, so
that is the interval between the roundings of the bound's two ends)."""
import ctypes
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import decode as od

pytestmark = pytest.mark.gpu
U = 2.0 ** -24


@pytest.fixture(scope="module")
def ctx(dev):
    from paper_2501_16909_amd import coloc
    c = coloc.Context(0)
    yield c
    c.close()


def _t(x, dev):
    import torch
    return torch.from_numpy(np.require(x, requirements=["C", "W"])).to(dev)


def _bf16(x32):
    """(codes as int16 for the device, FP64 values for the oracle)."""
    c = oracle.f32_to_bf16(np.asarray(x32, np.float32))
    return c.view(np.int16), oracle.bf16_to_f64(c).reshape(np.shape(x32))


def _vals(t):
    return oracle.bf16_to_f64(t.cpu().numpy().view(np.uint16)).reshape(tuple(t.shape))


def _assert_bf16_within(got, exact, eps, what):
    lo = od.q_bf16(exact - eps)
    hi = od.q_bf16(exact + eps)
    bad = ~((got >= lo) & (got <= hi))
    assert not bad.any(), (what, int(bad.sum()), got[bad][:4], exact[bad][:4], np.asarray(eps * np.ones_like(exact))[bad][:4])


# ---------------------------------------------------------------- RMSNorm
@pytest.mark.parametrize("rows,n", [(1, 4), (3, 516), (5, 4096), (2, 14336)])
def test_rmsnorm_matches_oracle(ctx, dev, rows, n):
    x = synth.uniform_affine_f32(synth.seed_for(5, 900), rows * n, 3.0).reshape(rows, n)
    gc, gv = _bf16(synth.uniform_affine_f32(synth.seed_for(5, 901), n, 0.25, 1.0))
    y = ctx.rmsnorm_bf16(_t(x, dev), _t(gc, dev), 1e-5)
    exact = od.rmsnorm(x.astype(np.float64), gv, 1e-5)
    # FP32: sum of n squares (n u), square root and reciprocal, two products
    _assert_bf16_within(_vals(y), exact, (n / 2 + 6) * U * np.abs(exact), "rmsnorm")


# ------------------------------------------------------------------- GEMV
@pytest.mark.parametrize("rows,k,batch", [(1, 8, 1), (7, 520, 3), (33, 4104, 8), (4101, 4096, 1),
                                          (300, 16392, 1), (64, 2056, 8), (257, 14336, 5), (5, 8, 8),
                                          (1000, 4096, 2), (130, 4096, 7)])
@pytest.mark.parametrize("res", ["none", "add", "alias"])
def test_gemv_rows_matches_oracle(ctx, dev, rows, k, batch, res):
    import torch
    wc, wv = _bf16(synth.uniform_affine_f32(synth.seed_for(5, 910), rows * k, 1.0 / math.sqrt(k)).reshape(rows, k))
    vc, vv = _bf16(synth.uniform_f32(synth.seed_for(5, 911), batch * k).reshape(batch, k))
    r = synth.uniform_f32(synth.seed_for(5, 912), batch * rows).reshape(batch, rows)
    W, V = _t(wc, dev), _t(vc, dev)
    if res == "none":
        out = ctx.gemv_bf16_rows(W, V)
        base = np.zeros((batch, rows))
    elif res == "add":
        out = ctx.gemv_bf16_rows(W, V, res=_t(r, dev))
        base = r.astype(np.float64)
    else:
        buf = _t(r, dev)
        out = ctx.gemv_bf16_rows(W, V, res=buf, out=buf)
        assert out.data_ptr() == buf.data_ptr()
        base = r.astype(np.float64)
    got = out.cpu().numpy().astype(np.float64)
    exact = vv @ wv.T + base
    bound = oracle.accumulation_bound(k + 1, np.abs(vv) @ np.abs(wv).T + np.abs(base), 2.0 ** -23)
    err = np.abs(got - exact)
    assert np.all(err <= bound), (float((err / np.maximum(bound, 1e-300)).max()),)
    torch.cuda.synchronize()


# ------------------------------------------------------------ RoPE + cache
@pytest.mark.parametrize("d,nq,nkv,base", [(128, 4, 2, 500000.0), (256, 2, 2, 10000.0), (128, 16, 1, 10000.0)])
def test_rope_append_matches_oracle(ctx, dev, d, nq, nkv, base):
    import torch
    batch, max_ctx = 3, 97
    pos = [0, 50, 96]
    heads = nq + 2 * nkv
    qkv = synth.uniform_affine_f32(synth.seed_for(5, 920), batch * heads * d, 2.0).reshape(batch, heads, d)
    kc0, _ = _bf16(synth.uniform_f32(synth.seed_for(5, 921), batch * nkv * max_ctx * d))
    vc0, _ = _bf16(synth.uniform_f32(synth.seed_for(5, 922), batch * nkv * max_ctx * d))
    kdev, vdev = _t(kc0, dev), _t(vc0, dev)
    q_out = torch.empty((batch, nq, d), dtype=torch.float32, device=dev)
    ctx.rope_append(_t(qkv, dev), pos, nq, nkv, d, max_ctx, base, q_out, kdev, vdev)
    qg = q_out.cpu().numpy().astype(np.float64)
    kg = _vals(kdev).reshape(batch, nkv, max_ctx, d)
    vg = _vals(vdev).reshape(batch, nkv, max_ctx, d)
    k_before = oracle.bf16_to_f64(kc0.view(np.uint16)).reshape(batch, nkv, max_ctx, d)
    v_before = oracle.bf16_to_f64(vc0.view(np.uint16)).reshape(batch, nkv, max_ctx, d)
    x = qkv.astype(np.float64)
    h = d // 2
    for b, p in enumerate(pos):
        pair = lambda a: np.concatenate([np.abs(a[..., :h]) + np.abs(a[..., h:])] * 2, axis=-1)
        want_q = od.rope(x[b, :nq], p, base)
        # FP32: cosine and sine rounded, two products and a sum per output
        assert np.all(np.abs(qg[b] - want_q) <= 6 * U * pair(x[b, :nq])), (b, p)
        want_k = od.rope(x[b, nq:nq + nkv], p, base)
        _assert_bf16_within(kg[b, :, p], want_k, 6 * U * pair(x[b, nq:nq + nkv]), "k cache")
        assert np.array_equal(vg[b, :, p], od.q_bf16(x[b, nq + nkv:]))
        keep = np.ones(max_ctx, bool)
        keep[p] = False
        assert np.array_equal(kg[b][:, keep], k_before[b][:, keep])
        assert np.array_equal(vg[b][:, keep], v_before[b][:, keep])


# -------------------------------------------------------------- attention
@pytest.mark.parametrize("d,nq,nkv,pos,qscale", [
    (128, 8, 2, [0, 63, 64, 199], 1.0),
    (128, 8, 2, [130, 5, 199, 64], 8.0),      # sharp softmax
    (256, 2, 2, [1, 199], 1.0),
    (128, 16, 1, [199], 2.0),                  # group of 16 waves
    (128, 4, 4, [0], 1.0)])
def test_attention_matches_oracle(ctx, dev, d, nq, nkv, pos, qscale):
    batch, max_ctx = len(pos), 200
    q = synth.uniform_affine_f32(synth.seed_for(5, 930), batch * nq * d, qscale).reshape(batch, nq, d)
    kc, kv = _bf16(synth.uniform_f32(synth.seed_for(5, 931), batch * nkv * max_ctx * d))
    vc, vv = _bf16(synth.uniform_f32(synth.seed_for(5, 932), batch * nkv * max_ctx * d))
    kv = kv.reshape(batch, nkv, max_ctx, d)
    vv = vv.reshape(batch, nkv, max_ctx, d)
    out = ctx.attention_decode(_t(q, dev), _t(kc, dev), _t(vc, dev), pos, nq, nkv, d, max_ctx)
    got = _vals(out).reshape(batch, nq, d)
    for b, p in enumerate(pos):
        want = od.attention_decode(q[b].astype(np.float64), kv[b, :, :p + 1], vv[b, :, :p + 1])
        # FP32 softmax: 64-term sums per chunk, then a merge over the chunks
        eps = (64 + (p // 64 + 1) + 8) * 2 * U * np.max(np.abs(vv[b, :, :p + 1]))
        _assert_bf16_within(got[b], want, eps, f"attention b={b} pos={p}")


# ------------------------------------------------------------------- SiLU
def test_silu_mul_matches_oracle(ctx, dev):
    batch, f = 3, 1000
    gu = synth.uniform_affine_f32(synth.seed_for(5, 940), batch * 2 * f, 6.0).reshape(batch, 2 * f)
    h = ctx.silu_mul_bf16(_t(gu, dev), f)
    g64 = gu.astype(np.float64)
    want = od.silu_mul(g64[:, :f], g64[:, f:])
    _assert_bf16_within(_vals(h), want, 8 * U * np.abs(want) + 1e-30, "silu")


# ------------------------------------------------------- fused GEMV forms
def _fused_inputs(dev, rows, k, batch, seed):
    wc, _ = _bf16(synth.uniform_affine_f32(seed, rows * k, 1.0 / math.sqrt(k)).reshape(rows, k))
    x = synth.uniform_affine_f32(seed + 1, batch * k, 2.0).reshape(batch, k)
    gc, _ = _bf16(synth.uniform_affine_f32(seed + 2, k, 0.25, 1.0))
    vc, _ = _bf16(synth.uniform_f32(seed + 3, batch * k).reshape(batch, k))
    return _t(wc, dev), _t(x, dev), _t(gc, dev), _t(vc, dev)


@pytest.mark.parametrize("batch", [1, 3, 8])
@pytest.mark.parametrize("k", [512, 4104])
def test_fused_gemv_equals_unfused_composition(ctx, dev, batch, k):
    """Every fused form gives, bit for bit, what the separate kernels give
    (RMS norm, then GEMV, then SiLU or rotary/cache append): same
    arithmetic, same summation order.  The separate kernels are pinned to
    the oracle above."""
    import torch
    eps = 1e-5
    # norm + plain (+ residual)
    w, x, g, v = _fused_inputs(dev, 300, k, batch, synth.seed_for(5, 960))
    res = _t(synth.uniform_f32(synth.seed_for(5, 965), batch * 300).reshape(batch, 300), dev)
    out = torch.empty((batch, 300), dtype=torch.float32, device=dev)
    ctx.fused_gemv(w, "plain", x=x, g=g, eps=eps, res=res, out=out)
    xn = ctx.rmsnorm_bf16(x, g, eps)
    ref = ctx.gemv_bf16_rows(w, xn, res=res)
    assert torch.equal(out.view(torch.int32), ref.view(torch.int32))
    # norm + SiLU: rows = 2 ffn
    f = 260
    w2, _, _, _ = _fused_inputs(dev, 2 * f, k, batch, synth.seed_for(5, 970))
    h = torch.empty((batch, f), dtype=torch.int16, device=dev)
    ctx.fused_gemv(w2, "silu", x=x, g=g, eps=eps, h=h)
    gu = ctx.gemv_bf16_rows(w2, xn)
    assert torch.equal(h, ctx.silu_mul_bf16(gu, f))
    # BF16 input + SiLU
    ctx.fused_gemv(w2, "silu", v=v, h=h)
    assert torch.equal(h, ctx.silu_mul_bf16(ctx.gemv_bf16_rows(w2, v), f))
    # norm + rotary / cache append
    nq, nkv, d, max_ctx = 4, 2, 128, 70
    pos = [(7 * b + 3) % max_ctx for b in range(batch)]
    pos[-1] = max_ctx - 1
    rows = (nq + 2 * nkv) * d
    w3, _, _, _ = _fused_inputs(dev, rows, k, batch, synth.seed_for(5, 980))
    caches = []
    for _ in range(2):
        kc0, _ = _bf16(synth.uniform_f32(synth.seed_for(5, 985), batch * nkv * max_ctx * d))
        vc0, _ = _bf16(synth.uniform_f32(synth.seed_for(5, 986), batch * nkv * max_ctx * d))
        caches.append((_t(kc0, dev), _t(vc0, dev), torch.empty((batch, nq, d), dtype=torch.float32, device=dev)))
    (k1, v1, q1), (k2, v2, q2) = caches
    ctx.fused_gemv(w3, "rope", x=x, g=g, eps=eps, pos=pos, n_q=nq, n_kv=nkv, head_dim=d, max_ctx=max_ctx,
                   rope_base=500000.0, q_out=q1, k_cache=k1, v_cache=v1)
    qkv = ctx.gemv_bf16_rows(w3, xn)
    ctx.rope_append(qkv, pos, nq, nkv, d, max_ctx, 500000.0, q2, k2, v2)
    assert torch.equal(q1.view(torch.int32), q2.view(torch.int32))
    assert torch.equal(k1, k2) and torch.equal(v1, v2)


def test_fused_gemv_rejects_bad_arguments(ctx, dev):
    import torch
    from paper_2501_16909_amd import coloc
    w, x, g, v = _fused_inputs(dev, 16, 64, 2, synth.seed_for(5, 990))
    out = torch.empty((2, 16), dtype=torch.float32, device=dev)
    with pytest.raises(coloc.CiError):            # odd row count for SiLU
        ctx.fused_gemv(w[:15], "silu", v=v, h=out)
    with pytest.raises(coloc.CiError):            # ROPE rows do not match the heads
        ctx.fused_gemv(w, "rope", v=v, pos=[0, 1], n_q=1, n_kv=1, head_dim=128, max_ctx=4, q_out=out,
                       k_cache=out, v_cache=out)
    lib = coloc.load_library()
    assert lib.ci_fused_gemv(ctx.handle, None, None) == 1
    a = coloc.GemvArgs()                          # neither a BF16 nor an FP32 input
    a.w, a.rows, a.k, a.batch, a.out = w.data_ptr(), 16, 64, 2, out.data_ptr()
    assert lib.ci_fused_gemv(ctx.handle, ctypes.byref(a), None) == 1
    a.v, a.batch = v.data_ptr(), 9                # batch beyond 8
    assert lib.ci_fused_gemv(ctx.handle, ctypes.byref(a), None) == 1


# -------------------------------------------------------------- whole step
def _host_inputs(cfg, seed):
    """Oracle-side inputs: the same seeded streams, rounded to BF16 on the
    host."""
    layers = [dict() for _ in range(cfg["layers"])]
    final, extra, codes = {}, {}, {}
    for name, layer, sd, n, scale, offset in synth.decode_tensor_specs(cfg, seed):
        x = synth.uniform_affine_f32(sd, n, scale, offset)
        if name == "x_in":
            extra[name] = x.reshape(cfg["batch"], cfg["hidden"])
            continue
        c = oracle.f32_to_bf16(x)
        v = oracle.bf16_to_f64(c)
        codes[(name, layer)] = c
        if name in ("k_cache", "v_cache"):
            extra[name] = v.reshape(cfg["layers"], cfg["batch"], cfg["n_kv"], cfg["max_ctx"], cfg["head_dim"])
            continue
        shape = {"g_attn": (-1,), "g_mlp": (-1,), "g_final": (-1,), "w_qkv": (-1, cfg["hidden"]),
                 "w_o": (cfg["hidden"], -1), "w_gu": (-1, cfg["hidden"]), "w_down": (cfg["hidden"], -1),
                 "w_lm": (-1, cfg["hidden"])}[name]
        v = v.reshape(shape) if n else np.zeros((0, cfg["hidden"]))
        if layer >= 0:
            layers[layer][name] = v
        else:
            final["g" if name == "g_final" else name] = v
    return layers, final, extra, codes


def _check_step(ctx, dev, cfg, pos, seed, tol):
    from paper_2501_16909_amd import coloc
    model = coloc.DecodeModel(ctx, cfg, pos, seed)
    layers, final, extra, codes = _host_inputs(cfg, seed)
    # the device drew and rounded the same inputs, bit for bit
    for (name, layer), c in codes.items():
        if name in ("k_cache", "v_cache"):
            got = getattr(model, name).cpu().numpy().view(np.uint16)
        else:
            got = model.tensor(name, layer).cpu().numpy().view(np.uint16)
        assert np.array_equal(got, c), (name, layer)
    assert np.array_equal(model.x_in.cpu().numpy(), extra["x_in"])
    r1 = ctx.decode_step(model)
    r2 = ctx.decode_step(model)
    assert r1["checksum_bits"] == r2["checksum_bits"]    # idempotent step
    kc, vc = extra["k_cache"], extra["v_cache"]
    want = od.decode_step(dict(cfg), layers, final, kc, vc, extra["x_in"], np.array(pos))
    got_x = model.x_out.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(got_x - want["x_out"]) / np.linalg.norm(want["x_out"])
    assert rel <= tol, ("x_out", rel)
    if cfg["vocab"]:
        got_l = model.logits.cpu().numpy().astype(np.float64)
        rel_l = np.linalg.norm(got_l - want["logits"]) / np.linalg.norm(want["logits"])
        assert rel_l <= tol, ("logits", rel_l)
    # the appended cache entries
    kd = _vals(model.k_cache).reshape(kc.shape)
    vd = _vals(model.v_cache).reshape(vc.shape)
    for b, p in enumerate(pos):
        for arr_d, arr_o in ((kd, kc), (vd, vc)):
            a, o = arr_d[:, b, :, p], arr_o[:, b, :, p]
            assert np.linalg.norm(a - o) <= tol * np.linalg.norm(o)
    used = [k for k, v in r1["kernel_ns"].items() if v > 0]
    expect = 6 + (1 if cfg["vocab"] else 0)
    assert len(used) == expect, r1["kernel_ns"]
    assert r1["step_ns"] >= 0.95 * sum(r1["kernel_ns"].values())
    return model, r1, rel


SMALL = dict(hidden=512, n_q=4, n_kv=2, head_dim=128, ffn=1032, vocab=1000, layers=2, batch=3,
             max_ctx=300, eps=1e-5, rope_base=500000.0)


def test_decode_step_small_model_matches_oracle(ctx, dev):
    """Two layers, three sequences at positions 0, 150 and 299 (ragged,
    first and last cache entry).  Tolerance: each of the step's BF16
    roundings can land one code away when FP32 and FP64 straddle a
    rounding boundary (2^-8 relative on that element, rarely); normwise the
    step stays far inside 2^-10, while a wrong index, head or term is an
    O(1) error."""
    _check_step(ctx, dev, SMALL, [0, 150, 299], synth.seed_for(5, 0), 2.0 ** -10)


def test_decode_step_group_sizes_and_head_dim_256(ctx, dev):
    cfg = dict(SMALL, n_q=8, n_kv=1, head_dim=256, layers=1, batch=1, max_ctx=129, vocab=0, hidden=264,
               ffn=520)
    _check_step(ctx, dev, cfg, [128], synth.seed_for(5, 100), 2.0 ** -10)


def test_decode_step_rejects_bad_positions(ctx, dev):
    from paper_2501_16909_amd import coloc
    model = coloc.DecodeModel(ctx, dict(SMALL, layers=1, batch=2, vocab=0), [0, 1], synth.seed_for(5, 200))
    model.set_positions([0, 300])
    with pytest.raises(coloc.CiError) as ei:
        ctx.decode_step(model)
    assert ei.value.status == 1
    model.set_positions([-1, 3])
    with pytest.raises(coloc.CiError):
        ctx.decode_step(model)


LLAMA_LAYER = dict(hidden=4096, n_q=32, n_kv=8, head_dim=128, ffn=14336, vocab=1024, layers=1, batch=2,
                   max_ctx=4096, eps=1e-5, rope_base=500000.0)


def test_decode_step_full_width_llama_layer(ctx, dev):
    """One Llama-3.1-8B layer at full width with a 4096-entry cache, the
    shape every layer of the benchmark's step has."""
    _, r, rel = _check_step(ctx, dev, LLAMA_LAYER, [4095, 1000], synth.seed_for(5, 300), 2.0 ** -10)
    print(f"full-width layer: rel err {rel:.2e}, step {r['step_ns'] / 1e3:.1f} us")


def test_decode_step_graph_and_plain_modes_match_timed(ctx, dev):
    """The same step launched with per-kernel events, without events, and
    replayed as a captured HIP graph gives bit-identical outputs; graph
    replays are interleaved with eager steps, and new positions within the
    same 64-entry bucket reuse the graph with the positions as data.  (A
    step appends to the cache, so the second position set lies past the
    first in every sequence: the first never reads what the second wrote.)"""
    from paper_2501_16909_amd import coloc
    cfg = dict(SMALL, layers=2, batch=2)
    model = coloc.DecodeModel(ctx, cfg, [100, 37], synth.seed_for(5, 500))
    ref = {}
    for pos in ([100, 37], [101, 38]):
        model.set_positions(pos)
        model.set_flags(coloc.DECODE_KERNEL_TIMES)
        ref[tuple(pos)] = ctx.decode_step(model)["checksum_bits"]
    for rep in range(3):
        for pos in ([100, 37], [101, 38]):
            model.set_positions(pos)
            model.set_flags(coloc.DECODE_GRAPH)
            r = ctx.decode_step(model)
            assert r["checksum_bits"] == ref[tuple(pos)], (rep, pos)
            assert all(v == 0 for v in r["kernel_ns"].values()) and r["step_ns"] > 0
            model.set_flags(0)
            assert ctx.decode_step(model)["checksum_bits"] == ref[tuple(pos)]
    model.set_flags(coloc.DECODE_KERNEL_TIMES | coloc.DECODE_GRAPH)
    with pytest.raises(coloc.CiError):
        ctx.decode_step(model)


def test_measure_decode_alone_and_colocated(ctx, dev):
    import torch
    from paper_2501_16909_amd import coloc
    cfg = dict(SMALL, layers=2, batch=1, vocab=1000)
    model = coloc.DecodeModel(ctx, cfg, [200], synth.seed_for(5, 400))
    n = 1 << 24
    b = torch.empty(n, dtype=torch.float32, device=dev)
    c, a = torch.empty_like(b), torch.empty_like(b)
    synth.device_fill_uniform_f32(b.data_ptr(), n, synth.seed_for(5, 950))
    synth.device_fill_uniform_f32(c.data_ptr(), n, synth.seed_for(5, 951))
    torch.cuda.synchronize()
    hbm = [dict(src0=b, src1=c, dst=a, n=n)]
    # per-kernel breakdown: launches with their own events
    for cell in ctx.measure_decode(model, ["hbm"], hbm, [0.0, 1.0], reps=5, warmups=2):
        assert cell["output_equal"] and cell["reps"] == 5 and not cell["timed_out"]
        assert cell["kernel_alone_ns"]["qkv"] > 0 and cell["kernel_col_ns"]["lm_head"] > 0
    # step times: the step replayed as a graph, so that host launch jitter
    # (which can leave gaps between a short step's kernels) stays out
    model.set_flags(coloc.DECODE_GRAPH)
    z, full = ctx.measure_decode(model, ["hbm"], hbm, [0.0, 1.0], reps=9, warmups=3)
    for cell in (z, full):
        assert cell["output_equal"] and cell["reps"] == 9 and not cell["timed_out"]
        assert cell["step_alone_p50"] > 0 and cell["step_alone_p90"] >= cell["step_alone_p50"]
        assert all(v == 0 for v in cell["kernel_alone_ns"].values())
    assert full["window_covered"] and full["ncu"] == 256
    assert full["step_col_p50"] > 1.05 * full["step_alone_p50"], full
    # the zero-intensity invariant, 1.00 +- 0.02, on a step long enough
    # (eight layers, a few hundred microseconds) for 31 counterbalanced
    # graph replays to settle the median
    long_model = coloc.DecodeModel(ctx, dict(SMALL, layers=8, batch=1, vocab=1000), [200],
                                   synth.seed_for(5, 410), flags=coloc.DECODE_GRAPH)
    z, = ctx.measure_decode(long_model, ["hbm"], hbm, [0.0], reps=31, warmups=10)
    assert z["output_equal"] and z["reps"] == 31
    assert abs(z["step_col_p50"] / z["step_alone_p50"] - 1.0) <= 0.02, z
    print(f"decode zero-intensity cell: {z['step_col_p50'] / z['step_alone_p50']:.4f} "
          f"(step {z['step_alone_p50'] / 1e3:.1f} us)")
    # disjoint halves: the graph replays on the victim's CU-masked queue
    half, = ctx.measure_decode(model, ["hbm"], hbm, [0.5], reps=5, warmups=2, placement="disjoint")
    assert half["output_equal"] and half["window_covered"] and half["ncu"] == 128, half
    assert half["step_alone_p50"] > 0 and half["step_col_p50"] > 0
