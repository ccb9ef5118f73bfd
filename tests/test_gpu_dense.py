"""GPU parity of the dense victims and the quantizers against the oracle:
quantised codes bit for bit, GEMM/GEMV within the FP32-accumulation bound of
an FP64 product of the same quantised inputs, outputs identical alone and
colocated."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(dev):
    from paper_2501_16909_amd import coloc
    c = coloc.Context(0)
    yield c
    c.close()


def _t(x, dev):
    import torch
    return torch.from_numpy(np.require(x, requirements=["C", "W"])).to(dev)


# ------------------------------------------------------------- quantizers
def test_bf16_quantizer_bit_exact(ctx, dev):
    x = np.concatenate([synth.normal_f32(41, 1 << 20),
                        np.array([0x3F808000, 0x3F818000, 0x7F7FFFFF, 0xFF7FFFFF, 0x7F800000,
                                  0x00000001, 0x80000000, 0x7FC00000], np.uint32).view(np.float32)])
    codes, _ = ctx.quantize(_t(x, dev), "bf16")
    got = codes.cpu().numpy().view(np.uint16)
    want = oracle.f32_to_bf16(x)
    nan = np.isnan(x)
    assert np.array_equal(got[~nan], want[~nan])
    assert np.all((got[nan] & 0x7FC0) == 0x7FC0)


@pytest.mark.parametrize("scale", [1.0, 1e-3, 300.0])
def test_fp8_quantizer_bit_exact(ctx, dev, scale):
    x = (synth.normal_f32(42, (1 << 20) + 3) * np.float32(scale)).astype(np.float32)
    x[:4] = [0.0, -0.0, x[4] * 1e-6, -x[5]]
    codes, s = ctx.quantize(_t(x, dev), "fp8")
    want, ws = oracle.quantize_fp8(x)
    assert s == ws
    assert np.array_equal(codes.cpu().numpy(), want)


def test_fp8_quantizer_every_e4m3_value_and_midpoint(ctx, dev):
    t = oracle.e4m3_table()
    fin = np.sort(np.unique(t[np.isfinite(t)]))
    mids = ((fin[1:] + fin[:-1]) / 2).astype(np.float32)
    # amax = 448 makes the scaling step exact (inv = 1)
    x = np.concatenate([fin.astype(np.float32), mids, -mids, np.array([448.0], np.float32)])
    codes, s = ctx.quantize(_t(x, dev), "fp8")
    want, ws = oracle.quantize_fp8(x)
    assert s == ws == 1.0
    assert np.array_equal(codes.cpu().numpy(), want)


# ------------------------------------------------------------------- GEMM
# Error bounds per input type.  FP32 and BF16: gamma_{K+1} * |A||B|^T with
# unit 2^-23 (faithful FP32 accumulation; the characterisation test below
# measures the FP32 and BF16 instructions well inside it).  FP8: the matrix
# core aligns each group of 8 products to the group's largest exponent and
# keeps 13 bits below it (characterised by test_mfma_fp8_accumulation_model
# on seeded adversarial tiles); oracle.mfma_fp8_error_bound turns that into
# a per-entry bound.
UNIT = {"f32": 2.0 ** -23, "bf16": 2.0 ** -23}


def _gemm_bound(dtype, qa, qb, fa, fb, scale, rows=None, cols=None):
    """Bound on |computed - exact| for the entries (rows[k], cols[k]) (all
    entries when rows is None); qa / qb hold the operands' codes (FP8) and
    fa / fb their values."""
    k = fa.shape[1]
    if dtype != "fp8":
        if rows is None:
            return scale * oracle.accumulation_bound(k + 1, oracle.gemm_abs_f64(fa, fb), UNIT[dtype])
        absw = oracle.gemm_entries_f64(np.abs(fa), np.abs(fb), rows, cols)
        return scale * oracle.accumulation_bound(k + 1, absw, UNIT[dtype])
    if rows is None:
        m, n = fa.shape[0], fb.shape[0]
        rows = np.repeat(np.arange(m), n)
        cols = np.tile(np.arange(n), m)
        out = np.empty(m * n)
        for lo in range(0, m * n, 4096):
            out[lo:lo + 4096] = oracle.mfma_fp8_error_bound(qa[rows[lo:lo + 4096]], qb[cols[lo:lo + 4096]], scale)
        return out.reshape(m, n)
    return oracle.mfma_fp8_error_bound(qa[rows], qb[cols], scale)
def _gemm_inputs(dtype, m, n, k, seed):
    a = synth.normal_f32(seed, m * k).reshape(m, k)
    b = synth.normal_f32(seed + 1, n * k).reshape(n, k)
    return a, b


def _quantise_host(x, dtype):
    if dtype == "f32":
        return x, x.astype(np.float64), 1.0
    if dtype == "bf16":
        q = oracle.f32_to_bf16(x)
        return q.view(np.int16), oracle.bf16_to_f64(q), 1.0
    q, s = oracle.quantize_fp8(x)
    return q, oracle.e4m3_to_f64(q), float(s)


def _dequant(codes, dtype):
    if dtype == "f32":
        return codes.astype(np.float64)
    if dtype == "bf16":
        return oracle.bf16_to_f64(codes.view(np.uint16))
    return oracle.e4m3_to_f64(codes)


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
@pytest.mark.parametrize("m,n,k", [(128, 128, 128), (256, 384, 512), (200, 130, 64), (1, 1, 16),
                                   (512, 512, 1040), (1000, 777, 336),
                                   (4100, 4000, 336),     # large tiles, ragged edges
                                   (4100, 4000, 64),      # LDS ring: 4 / 2 / 1 stages (f32 / bf16 / fp8)
                                   (4100, 4000, 192)])    # LDS ring: 12 / 6 / 3 stages
def test_gemm_matches_oracle(ctx, dev, dtype, m, n, k):
    import torch
    a, b = _gemm_inputs(dtype, m, n, k, 1000 + m + n + k)
    qa, fa, sa = _quantise_host(a, dtype)
    qb, fb, sb = _quantise_host(b, dtype)
    out = torch.full((m, n), float("nan"), dtype=torch.float32, device=dev)
    d = ctx.gemm_desc(_t(qa, dev), _t(qb, dev), out, dtype, m, n, k, sa, sb)
    r = ctx.victim_run(d)
    got = out.cpu().numpy().astype(np.float64)
    want = sa * sb * oracle.gemm_f64(fa, fb)
    if dtype == "fp8" and m * n > 1 << 18:      # the per-entry FP8 bound on a fixed sample
        idx = synth.words(77 + k, 8192)
        rows = (idx % np.uint64(m)).astype(np.int64)
        cols = ((idx >> np.uint64(32)) % np.uint64(n)).astype(np.int64)
        err = np.abs(got[rows, cols] - want[rows, cols])
        bound = _gemm_bound(dtype, qa, qb, fa, fb, sa * sb, rows, cols)
        print(f"{dtype} {m}x{n}x{k}: max err/bound {float((err / np.maximum(bound, 1e-300)).max()):.3g} (sampled)")
        assert np.all(err <= bound)
        assert r.checksum_bits == oracle.bitsum_u32(out.cpu().numpy())
        return
    bound = _gemm_bound(dtype, qa, qb, fa, fb, sa * sb)
    err = np.abs(got - want)
    print(f"{dtype} {m}x{n}x{k}: max err/bound {float((err / np.maximum(bound, 1e-300)).max()):.3g}")
    assert np.all(err <= bound)
    assert r.checksum_bits == oracle.bitsum_u32(out.cpu().numpy())


def test_gemm_identity_is_exact(ctx, dev):
    import torch
    n = 256
    a = oracle.f32_to_bf16(synth.normal_f32(7, n * n)).reshape(n, n)
    eye = oracle.f32_to_bf16(np.eye(n, dtype=np.float32))
    out = torch.empty((n, n), dtype=torch.float32, device=dev)
    ctx.victim_run(ctx.gemm_desc(_t(a.view(np.int16), dev), _t(eye.view(np.int16), dev), out, "bf16", n, n, n))
    assert np.array_equal(out.cpu().numpy(), oracle.bf16_to_f64(a).astype(np.float32))


def test_gemm_4096_sampled(ctx, dev):
    """The sweep victim at full size: M = N = K = 4096 BF16, sampled entries
    checked one dot product at a time."""
    import torch
    m = n = k = 4096
    a = synth.normal_f32(synth.seed_for(2, synth.BUF_GEMM_A), m * k).reshape(m, k)
    b = synth.normal_f32(synth.seed_for(2, synth.BUF_GEMM_B), n * k).reshape(n, k)
    ta, tb = _t(a, dev), _t(b, dev)
    qa, _ = ctx.quantize(ta, "bf16")
    qb, _ = ctx.quantize(tb, "bf16")
    out = torch.empty((m, n), dtype=torch.float32, device=dev)
    r1 = ctx.victim_run(ctx.gemm_desc(qa, qb, out, "bf16", m, n, k))
    r2 = ctx.victim_run(ctx.gemm_desc(qa, qb, out, "bf16", m, n, k))
    assert r1.checksum_bits == r2.checksum_bits            # deterministic
    ha, hb = oracle.f32_to_bf16(a), oracle.f32_to_bf16(b)
    assert np.array_equal(qa.cpu().numpy().view(np.uint16), ha)
    idx = synth.words(99, 2048)
    rows = (idx % np.uint64(m)).astype(np.int64)
    cols = ((idx >> np.uint64(32)) % np.uint64(n)).astype(np.int64)
    fa, fb = oracle.bf16_to_f64(ha), oracle.bf16_to_f64(hb)
    want = oracle.gemm_entries_f64(fa, fb, rows, cols)
    absw = oracle.gemm_entries_f64(np.abs(fa), np.abs(fb), rows, cols)
    got = out.cpu().numpy()[rows, cols]
    assert np.all(np.abs(got - want) <= oracle.accumulation_bound(k + 1, absw, 2.0 ** -23))
    tflops = 2.0 * m * n * k / r2.time_ns / 1e3
    print(f"bf16 gemm 4096^3: {r2.time_ns/1e3:.1f} us, {tflops:.0f} TFLOP/s")


@pytest.fixture(scope="module")
def gemm8192_inputs():
    """Config 3's inputs: A and B of 8192 x 8192 from N(0, 1) in FP32."""
    n = 8192
    a = synth.normal_f32(synth.seed_for(3, synth.BUF_GEMM_A), n * n).reshape(n, n)
    b = synth.normal_f32(synth.seed_for(3, synth.BUF_GEMM_B), n * n).reshape(n, n)
    return a, b


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
def test_gemm_8192_precision_sampled(ctx, dev, gemm8192_inputs, dtype):
    """The precision workload at full size: M = N = K = 8192 from N(0, 1),
    quantised on the device (codes and scale equal to the oracle's
    quantiser), 4096 fixed-seed entries against the FP64 product of the
    quantised inputs within the dtype's bound, and the whole output bit for
    bit the same beside a running HBM stressor."""
    import torch
    a, b = gemm8192_inputs
    m = n = k = 8192
    ta, tb = _t(a, dev), _t(b, dev)
    if dtype == "f32":
        qa, qb, sa, sb = ta, tb, 1.0, 1.0
        ha, hb = a, b
    else:
        qa, sa = ctx.quantize(ta, dtype)
        qb, sb = ctx.quantize(tb, dtype)
        if dtype == "bf16":
            ha, hb = oracle.f32_to_bf16(a).view(np.int16), oracle.f32_to_bf16(b).view(np.int16)
        else:
            (ha, wsa), (hb, wsb) = oracle.quantize_fp8(a), oracle.quantize_fp8(b)
            assert (sa, sb) == (wsa, wsb)
        assert np.array_equal(qa.cpu().numpy(), ha) and np.array_equal(qb.cpu().numpy(), hb)
    del ta, tb
    out = torch.empty((m, n), dtype=torch.float32, device=dev)
    d = ctx.gemm_desc(qa, qb, out, dtype, m, n, k, sa, sb)
    r1 = ctx.victim_run(d)
    alone = out.cpu().numpy().copy()
    sbuf = [torch.empty(1 << 26, dtype=torch.float32, device=dev) for _ in range(3)]
    for t in sbuf[:2]:
        synth.device_fill_uniform_f32(t.data_ptr(), 1 << 26, 991)
    with ctx.stressor("hbm", 0.5, src0=sbuf[0], src1=sbuf[1], dst=sbuf[2], n=1 << 26) as st:
        r2 = ctx.victim_run(d)
    assert not st.report.timed_out
    assert r2.checksum_bits == r1.checksum_bits
    assert np.array_equal(out.cpu().numpy().view(np.uint32), alone.view(np.uint32))
    idx = synth.words(8192, 4096)
    rows = (idx % np.uint64(m)).astype(np.int64)
    cols = ((idx >> np.uint64(32)) % np.uint64(n)).astype(np.int64)
    fa, fb = _dequant(ha[rows], dtype), _dequant(hb[cols], dtype)
    pair = np.arange(4096)
    want = sa * sb * oracle.gemm_entries_f64(fa, fb, pair, pair)
    bound = _gemm_bound(dtype, ha[rows], hb[cols], fa, fb, sa * sb, pair, pair)
    got = alone[rows, cols].astype(np.float64)
    err = np.abs(got - want)
    ratio = float((err / np.maximum(bound, 1e-300)).max())
    absw = sa * sb * oracle.gemm_entries_f64(np.abs(fa), np.abs(fb), pair, pair)
    print(f"{dtype} gemm 8192^3: {r1.time_ns / 1e6:.2f} ms, {2.0 * m * n * k / r1.time_ns / 1e3:.0f} TFLOP/s; "
          f"max err/bound {ratio:.3g}; max err/(|A||B|^T) {float((err / absw).max()):.3g}; "
          f"normwise {float(np.linalg.norm(got - want) / np.linalg.norm(want)):.3g}")
    assert np.all(err <= bound)


def test_gemm_rejects_bad_k(ctx, dev):
    import torch
    from paper_2501_16909_amd import coloc
    a = torch.zeros((64, 12), dtype=torch.int16, device=dev)
    out = torch.empty((64, 64), dtype=torch.float32, device=dev)
    with pytest.raises(coloc.CiError) as ei:
        ctx.victim_run(ctx.gemm_desc(a, a, out, "bf16", 64, 64, 12))
    assert ei.value.status == 1


# ------------------------------------------------------------------- GEMV
@pytest.mark.parametrize("n,k,copies", [(1, 8, 1), (3, 64, 2), (1000, 4104, 1), (8192, 8192, 3)])
def test_gemv_matches_oracle(ctx, dev, n, k, copies):
    import torch
    w = oracle.f32_to_bf16(synth.normal_f32(synth.seed_for(2, synth.BUF_GEMV_W), n * k, sigma=0.02)).reshape(n, k)
    x = oracle.f32_to_bf16(synth.normal_f32(synth.seed_for(2, synth.BUF_GEMV_X), k))
    tw = _t(np.broadcast_to(w.view(np.int16), (copies, n, k)), dev)
    y = torch.empty(n, dtype=torch.float32, device=dev)
    d = ctx.gemv_desc(tw, _t(x.view(np.int16), dev), y, n, k, copies)
    fw, fx = oracle.bf16_to_f64(w), oracle.bf16_to_f64(x)
    want = oracle.gemv_f64(fw, fx)
    bound = oracle.accumulation_bound(k + 1, np.abs(fw) @ np.abs(fx), 2.0 ** -24)
    sums = set()
    for rep in range(copies + 1):                 # every weight copy in turn
        r = ctx.victim_run(d)
        got = y.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(got - want) <= bound)
        sums.add(r.checksum_bits)
    assert len(sums) == 1
    if n == 8192:
        gbs = n * k * 2 / r.time_ns
        print(f"gemv 8192^2: {r.time_ns/1e3:.1f} us, {gbs:.0f} GB/s")


def test_victims_identical_alone_and_colocated(ctx, dev):
    """Outputs are bit-identical with and without every kind of stressor."""
    import torch
    m = n = k = 1024
    a = oracle.f32_to_bf16(synth.normal_f32(5, m * k)).view(np.int16)
    b = oracle.f32_to_bf16(synth.normal_f32(6, n * k)).view(np.int16)
    out = torch.empty((m, n), dtype=torch.float32, device=dev)
    d = ctx.gemm_desc(_t(a, dev), _t(b, dev), out, "bf16", m, n, k)
    base = ctx.victim_run(d).checksum_bits
    win = _t(synth.u32(3, 8192).view(np.int32), dev)
    w2m = _t(synth.u32(4, 1 << 19).view(np.int32), dev)
    vout = torch.empty(256 * 4 * 256 * 8, dtype=torch.float32, device=dev)
    cells = ctx.measure_sensitivity(d, ["lds", "l2", "valu_f32", "occupancy"],
                                    [dict(src0=win), dict(src0=w2m, n=1 << 19), dict(dst=vout), dict()],
                                    [0.5, 1.0], reps=3, warmups=1)
    for c in cells:
        assert c["output_equal"], c
        assert c["window_covered"], c
        print(f"gemm1024 vs {c['resource']}@{c['intensity']}: slowdown {c['slowdown']:.2f}")
    assert ctx.victim_run(d).checksum_bits == base


def test_victim_enqueue_runs_back_to_back(ctx, dev):
    import torch
    n = (1 << 20) + 9
    b = synth.uniform_f32(61, n)
    c = synth.uniform_f32(62, n)
    tb, tc = _t(b, dev), _t(c, dev)
    ta = torch.zeros(n, dtype=torch.float32, device=dev)
    s = torch.cuda.Stream(device=dev)
    d = ctx.triad_desc(tb, tc, ta, passes=1)
    ctx.victim_enqueue(d, s, 5)
    s.synchronize()
    assert np.array_equal(ta.cpu().numpy().view(np.uint32), oracle.triad_f32(b, c).view(np.uint32))
    from paper_2501_16909_amd import coloc
    with pytest.raises(coloc.CiError):
        ctx.victim_enqueue(d, None, 1)
