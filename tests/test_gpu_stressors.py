"""GPU parity of every stressor kernel against the oracle, in the fixed-pass
form (exact work) and in the persistent form (work as reported)."""
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


# ------------------------------------------------------------ cache loops
@pytest.mark.parametrize("res,words,x,passes", [
    ("vl1d", 4096, 1.0, 7),            # 16 KiB
    ("l2", 1 << 19, 0.25, 2),          # 2 MiB
    ("l2", 1 << 19, 1.0, 3),
])
def test_cache_stressor_fixed(ctx, dev, res, words, x, passes):
    w = synth.u32(synth.seed_for(1, synth.BUF_CACHE), words)
    tw = _t(w.view(np.int32), dev)
    st = ctx.stressor(res, x, src0=tw, n=words, passes=passes)
    rep = st.stop()
    rec = st.records()
    assert rep.wg_reported == rep.grid and np.all(rec["work"] == passes)
    exp = oracle.cache_wg_expected(w, rec["work"])
    assert np.array_equal(rec["check"].astype(np.uint32), exp)
    assert rep.units == 4.0 * words * passes * rep.grid


@pytest.mark.parametrize("res,words", [("vl1d", 4096), ("l2", 1 << 19)])
def test_cache_stressor_persistent(ctx, dev, res, words):
    import time
    w = synth.u32(synth.seed_for(1, synth.BUF_CACHE), words)
    tw = _t(w.view(np.int32), dev)
    with ctx.stressor(res, 1.0, src0=tw, n=words) as st:
        time.sleep(0.02)
    rep = st.report
    rec = st.records()
    assert not rep.timed_out and rep.wg_reported == rep.grid
    assert np.all(rec["work"] > 0)
    assert np.all(rec["flags"] & 2)          # every group saw the stop flag
    exp = oracle.cache_wg_expected(w, rec["work"])
    assert np.array_equal(rec["check"].astype(np.uint32), exp)
    print(f"{res}: {rep.achieved/1e12:.2f} TB/s ({rep.pct_of_peak:.1f}% of peak) over "
          f"{rep.window_ns/1e6:.2f} ms")


# --------------------------------------------------- Infinity Cache (MALL)
def _mall_buffers(dev, n):
    b = synth.uniform_f32(synth.seed_for(1, synth.BUF_B2) + 7, n)
    c = synth.uniform_f32(synth.seed_for(1, synth.BUF_C2) + 7, n)
    sentinel = np.full(n, 0x7FC0DEAD, np.uint32)
    return b, c, _t(b, dev), _t(c, dev), _t(sentinel.view(np.float32), dev), sentinel


@pytest.mark.parametrize("mix,x,passes,n,chunk", [
    ("read", 1.0, 2, 1 << 24, 2),          # b and c: 128 MiB, 16 MiB per XCD slot
    ("triad", 0.5, 1, (1 << 23) + 7, 1),   # three arrays of 32 MiB, ragged tail
    ("copy", 0.25, 3, 1 << 20, 4),
    ("write", 1.0, 1, 1 << 22, 2),
])
def test_mall_stressor_fixed(ctx, dev, mix, x, passes, n, chunk):
    """The Infinity-Cache stressor streams a footprint that fits the MALL:
    outputs bit-exact against the oracle, the read checksum exact mod 2^32,
    every wave-chunk counted `passes` times."""
    from paper_2501_16909_amd import coloc
    b, c, tb, tc, ta, sentinel = _mall_buffers(dev, n)
    ops = {"read": dict(src0=tb, src1=tc), "triad": dict(src0=tb, src1=tc, dst=ta),
           "copy": dict(src0=tb, dst=ta), "write": dict(dst=ta)}[mix]
    rep = ctx.stressor("mall", x, n=n, passes=passes, chunk=chunk, knob=coloc.HBM_MIX[mix], **ops).stop()
    got = ta.cpu().numpy().view(np.uint32)
    if mix == "read":
        assert np.array_equal(got, sentinel)
        assert rep.checksum % 2 ** 32 == oracle.hbm_read_checksum(b, c, passes)
    elif mix == "triad":
        assert np.array_equal(got, oracle.triad_f32(b, c).view(np.uint32))
    elif mix == "copy":
        assert np.array_equal(got, oracle.hbm_copy(b))
    else:
        assert np.array_equal(got, oracle.hbm_write_pattern(n))
    assert rep.grid == 8 * round(32 * x) and rep.wg_reported == rep.grid and not rep.timed_out
    assert rep.work == passes * ((n + 256 * chunk - 1) // (256 * chunk))
    assert rep.units == oracle.hbm_bytes_per_element(mix) * n * passes
    print(f"mall {mix}: {rep.achieved / 1e12:.2f} TB/s ({rep.pct_of_peak:.1f} % of the ceiling)")


def test_mall_stressor_persistent(ctx, dev):
    """Persistent triad mix over three 32 MiB arrays: after a run that swept
    every range many times, every element holds the oracle's value (the
    sweeps rewrite the same values), and the reported units are 12 bytes per
    element of every wave-chunk processed."""
    import time
    from paper_2501_16909_amd import coloc
    n = 1 << 23
    b, c, tb, tc, ta, sentinel = _mall_buffers(dev, n)
    with ctx.stressor("mall", 1.0, src0=tb, src1=tc, dst=ta, n=n, knob=coloc.HBM_MIX["triad"]) as st:
        time.sleep(0.03)
    rep = st.report
    rec = st.records()
    assert not rep.timed_out and rep.wg_reported == rep.grid and np.all(rec["flags"] & 2)
    nch = n // 1024
    assert rep.work >= 2 * nch                      # at least two sweeps of every range
    assert rep.units == 12.0 * 1024 * rep.work
    assert np.array_equal(ta.cpu().numpy().view(np.uint32), oracle.triad_f32(b, c).view(np.uint32))
    print(f"mall triad persistent: {rep.achieved / 1e12:.2f} TB/s over {rep.window_ns / 1e6:.1f} ms")


@pytest.mark.parametrize("res,mix,n", [
    ("hbm", "triad", (1 << 25) + 3),    # ticket form, three 128 MiB arrays
    ("hbm", "read", 1 << 25),           # strided form
    ("mall", "copy", 1 << 22),
])
def test_stream_stressor_duty_cycle(ctx, dev, res, mix, n):
    """Duty-cycled streaming stressors do the same work with the same
    results and only idle between stretches of work: the launch takes longer
    as duty falls, and at a quarter duty stays within a small multiple of the
    full-rate launch (the idle periods do not compound across the
    work-group's barriers)."""
    import torch
    from paper_2501_16909_amd import coloc
    b, c, tb, tc, ta, sentinel = _mall_buffers(dev, n)
    ops = {"read": dict(src0=tb, src1=tc), "triad": dict(src0=tb, src1=tc, dst=ta),
           "copy": dict(src0=tb, dst=ta)}[mix]
    times, sums = {}, {}
    for duty in (100, 50, 25):
        ta.copy_(torch.from_numpy(sentinel.view(np.float32)).to(dev))
        rep = ctx.stressor(res, 1.0, n=n, passes=2, knob=coloc.HBM_MIX[mix], duty=duty, **ops).stop()
        assert not rep.timed_out and rep.wg_reported == rep.grid
        assert rep.units == oracle.hbm_bytes_per_element(mix) * n * 2
        times[duty], sums[duty] = rep.kernel_ns, rep.checksum
        got = ta.cpu().numpy().view(np.uint32)
        if mix == "read":
            assert np.array_equal(got, sentinel)
            assert rep.checksum % 2 ** 32 == oracle.hbm_read_checksum(b, c, 2)
        elif mix == "triad":
            assert np.array_equal(got, oracle.triad_f32(b, c).view(np.uint32))
        else:
            assert np.array_equal(got, oracle.hbm_copy(b))
    assert times[100] < times[50] < times[25], times
    assert times[25] < 12 * times[100], times
    print(f"{res} {mix} duty 100/50/25: " + ", ".join(f"{times[d] / 1e3:.0f} us" for d in (100, 50, 25)))


@pytest.mark.parametrize("res", ["hbm", "mall"])
def test_stream_stressor_persistent_fewer_chunks_than_slots(ctx, dev, res):
    """A persistent stream over 3 wave-chunks (ragged last one) leaves five
    of the eight XCD slots without a range: their work-groups hold until
    stopped, every work-group reports and saw the stop flag, and the output
    is the oracle's."""
    import time
    from paper_2501_16909_amd import coloc
    n = 2 * 256 + 100                       # wave-chunks of 256 elements (chunk = 1)
    b, c, tb, tc, ta, sentinel = _mall_buffers(dev, n)
    with ctx.stressor(res, 1.0, src0=tb, src1=tc, dst=ta, n=n, chunk=1, knob=coloc.HBM_MIX["triad"]) as st:
        time.sleep(0.02)
    rep = st.report
    rec = st.records()
    assert not rep.timed_out and rep.wg_reported == rep.grid and np.all(rec["flags"] & 2)
    assert rep.work >= 3 and rep.units == 12.0 * 256 * rep.work
    assert np.array_equal(ta.cpu().numpy().view(np.uint32), oracle.triad_f32(b, c).view(np.uint32))


# -------------------------------------------------------------------- LDS
@pytest.mark.parametrize("vec,stride,access", [(1, 1, 0), (1, 2, 0), (1, 32, 0), (2, 1, 0), (4, 1, 0), (4, 3, 0),
                                               (4, 1, 1), (1, 32, 1), (2, 5, 1)])
def test_lds_stressor_fixed(ctx, dev, vec, stride, access):
    """Copy (access 0) and load-only (access 1) forms: every work-group's
    checksum of the words it read matches the oracle, and the reported bytes
    count loads, plus stores for the copy."""
    w = synth.u32(synth.seed_for(1, synth.BUF_LDS), 8192)
    st = ctx.stressor("lds", 0.25, src0=_t(w.view(np.int32), dev), vec=vec, knob=stride, passes=3,
                      threads=256, wg_per_cu=2, access=access)
    rep = st.stop()
    rec = st.records()
    exp = oracle.lds_wg_expected(w, vec, stride, waves=4, passes=rec["work"])
    assert np.all(rec["work"] == 3)
    assert np.array_equal(rec["check"].astype(np.uint32), exp)
    assert rep.units == 3 * rep.grid * 4 * 64 * 8192 * 4 * (1 if access else 2)
    st = ctx.stressor("lds", 0.25, src0=_t(w.view(np.int32), dev), vec=vec, knob=stride, passes=2, access=access)
    rep = st.stop()   # default shape: 1024 threads (16 waves), one work-group per CU
    rec = st.records()
    assert np.array_equal(rec["check"].astype(np.uint32),
                          oracle.lds_wg_expected(w, vec, stride, waves=16, passes=rec["work"]))


def test_lds_load_persistent_and_rejections(ctx, dev):
    import time
    from paper_2501_16909_amd import coloc
    w = synth.u32(synth.seed_for(1, synth.BUF_LDS), 8192)
    tw = _t(w.view(np.int32), dev)
    with ctx.stressor("lds", 1.0, src0=tw, access=coloc.LDS_ACCESS["load"]) as st:
        time.sleep(0.02)
    rep = st.report
    rec = st.records()
    assert not rep.timed_out and np.all(rec["flags"] & 2) and np.all(rec["work"] > 0)
    assert np.array_equal(rec["check"].astype(np.uint32),
                          oracle.lds_wg_expected(w, 4, 1, waves=16, passes=rec["work"]))
    print(f"lds load-only: {rep.achieved / 1e12:.1f} TB/s, {rep.pct_of_peak:.1f} % of the load path")
    with pytest.raises(coloc.CiError) as ei:
        ctx.stressor("lds", 0.25, src0=tw, access=2)
    assert ei.value.status == 1
    with pytest.raises(coloc.CiError) as ei:
        ctx.stressor("valu_f32", 0.25, dst=tw, access=1)
    assert ei.value.status == 1


# ------------------------------------------------------------------- VALU
@pytest.mark.parametrize("ilp,iters,passes,x", [(1, 4096, 1, 0.125), (2, 100, 3, 0.25), (4, 4096, 2, 0.5),
                                                 (8, 4096, 1, 1.0), (8, 13, 1, 1 / 32)])
def test_valu_stressor_fixed(ctx, dev, ilp, iters, passes, x):
    import torch
    ncu = 8 * round(32 * x)
    threads = ncu * 4 * 256          # default: four 256-thread work-groups per CU
    out = torch.empty(threads * ilp, dtype=torch.float32, device=dev)
    a, b = 1 - 2.0 ** -12, 2.0 ** -12
    st = ctx.stressor("valu_f32", x, dst=out, knob=ilp, iters=iters, passes=passes, fa=a, fb=b)
    rep = st.stop()
    got = out.cpu().numpy().reshape(threads, ilp)
    sel = np.unique(np.concatenate([np.arange(0, threads, 97), [threads - 1]]))
    want = oracle.valu_outputs(sel, ilp, a, b, iters * passes)
    assert np.array_equal(got[sel].view(np.uint32), want.view(np.uint32))
    assert rep.units == 2.0 * threads * ilp * iters * passes


def test_valu_closed_form_counts(ctx, dev):
    """fa = 1, fb = 1 from x0: each chain adds exactly one per step."""
    import torch
    threads = 8 * 4 * 256
    out = torch.empty(threads * 4, dtype=torch.float32, device=dev)
    st = ctx.stressor("valu_f32", 1 / 32, dst=out, knob=4, iters=1000, passes=2, fa=1.0, fb=1.0)
    st.stop()
    x0 = oracle.valu_start_values(np.arange(threads), 4)
    assert np.array_equal(out.cpu().numpy().reshape(threads, 4), x0 + np.float32(2000))


# ------------------------------------------------------------------- MFMA
def _mfma_operands(dtype, kind):
    k = {"f32": 2, "bf16": 16, "fp8": 64}[dtype]
    if kind == "ones":
        a = np.ones((32, k), np.float32)
        b = np.ones((k, 32), np.float32)
    else:
        a = synth.normal_f32(synth.seed_for(3, synth.BUF_MFMA), 32 * k).reshape(32, k)
        b = synth.normal_f32(synth.seed_for(3, synth.BUF_MFMA) + 1, k * 32).reshape(k, 32)
    if dtype == "f32":
        return a, b, a, b
    if dtype == "bf16":
        qa, qb = oracle.f32_to_bf16(a), oracle.f32_to_bf16(b)
        return qa.view(np.int16), qb.view(np.int16), oracle.bf16_to_f64(qa), oracle.bf16_to_f64(qb)
    qa = oracle.f32_to_e4m3(np.clip(a, -448, 448))
    qb = oracle.f32_to_e4m3(np.clip(b, -448, 448))
    return qa, qb, oracle.e4m3_to_f64(qa), oracle.e4m3_to_f64(qb)


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
@pytest.mark.parametrize("kind", ["ones", "normal"])
def test_mfma_stressor_fixed(ctx, dev, dtype, kind):
    import torch
    da, db, fa, fb = _mfma_operands(dtype, kind)
    iters, passes, x, accs = 100, 2, 0.125, 4
    ncu = 8 * round(32 * x)
    waves = ncu * 2 * 4
    out = torch.empty(waves * accs * 1024, dtype=torch.float32, device=dev)
    st = ctx.stressor(f"mfma_{dtype}", x, src0=_t(da, dev), src1=_t(db, dev), dst=out,
                      knob=accs, iters=iters, passes=passes)
    rep = st.stop()
    tiles = out.cpu().numpy().reshape(waves * accs, 32, 32)
    total = iters * passes
    want = oracle.mfma_tile_expected(fa, fb, total)
    if kind == "ones":
        assert np.all(tiles == want), (dtype, np.unique(tiles)[:5])
    else:
        absprod = total * (np.abs(fa) @ np.abs(fb))
        k = fa.shape[1]
        # each step: k exact products summed in FP32, then added to |acc| <= absprod.
        # The matrix core's internal rounding is not specified: the bound takes
        # faithful rounding (error below one ulp, u = 2^-23), which covers
        # round-to-nearest (2^-24) as well.
        unit = 2.0 ** -20 if dtype == "fp8" else 2.0 ** -23   # see the GEMM tests
        bound = oracle.accumulation_bound(k + total, absprod, unit_roundoff=unit)
        err = np.abs(tiles - want[None])
        print(f"{dtype}: max err/bound = {float((err / bound[None]).max()):.3f}")
        assert np.all(err <= bound[None]), (dtype, float(err.max()), float(bound.max()))
        assert np.all(tiles == tiles[0:1])   # every wave and accumulator agree bit for bit
    assert rep.units == waves * accs * total * 2.0 * 32 * 32 * fa.shape[1]


# ---------------------------------------------------------- pointer chase
@pytest.mark.parametrize("n,chains,hops,passes,x", [(1 << 12, 1, 4096, 1, 1 / 32),
                                                    (1 << 20, 4, 100, 3, 0.25),
                                                    (1 << 24, 8, 64, 1, 1.0)])
def test_chase_stressor_fixed(ctx, dev, n, chains, hops, passes, x):
    import torch
    nxt = synth.random_cycle_u32(synth.seed_for(1, synth.BUF_CHASE), n)
    ncu = 8 * round(32 * x)
    q = ncu * 256 * chains           # default: one 256-thread work-group per CU
    end = torch.empty(q, dtype=torch.int32, device=dev)
    st = ctx.stressor("ptrchase", x, src0=_t(nxt.view(np.int32), dev), n=n, dst=end, knob=chains,
                      iters=hops, passes=passes)
    rep = st.stop()
    starts = oracle.chase_starts(q, n)
    sel = np.unique(np.concatenate([np.arange(0, q, max(1, q // 2000)), [q - 1]]))
    want = oracle.chase_u32(nxt, starts[sel], hops * passes)
    got = end.cpu().numpy().view(np.uint32)[sel]
    assert np.array_equal(got, want)
    if n == 4096 and hops * passes == n:
        assert np.array_equal(got, starts[sel].astype(np.uint32))   # a full cycle returns
    assert rep.units == q // chains * chains * hops * passes


# --------------------------------------------------------- dispatch / hog
def test_dispatch_counts_every_workgroup(ctx, dev):
    import torch
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    st = ctx.stressor("dispatch", 1.0, dst=cnt, iters=1000000, passes=2)
    rep = st.stop()
    assert int(cnt.item()) == 2000000
    assert rep.units == 2e6
    st = ctx.stressor("dispatch", 0.5, iters=1000000, passes=1)   # empty kernel, timing form
    rep = st.stop()
    assert rep.kernel_ns > 0


def test_dispatch_persistent_feeder(ctx, dev):
    import time
    import torch
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    with ctx.stressor("dispatch", 1.0, dst=cnt, iters=100000) as st:
        time.sleep(0.05)
    rep = st.report
    assert int(cnt.item()) == rep.units and rep.units >= 100000
    print(f"dispatch: {rep.units/ (rep.kernel_ns*1e-9) / 1e6:.0f} M WG/s")


def test_occupancy_hog_holds_cus(ctx, dev):
    import time
    with ctx.stressor("occupancy", 0.5, knob=64) as st:
        time.sleep(0.01)
    rep = st.report
    rec = st.records()
    assert rep.wg_reported == rep.grid == 128 and rep.distinct_cus >= 64
    assert np.all(rec["flags"] & 2) and np.all(rec["work"] > 0)
    assert np.all(rec["check"] == 64 * 1024 // 4 - 1)


def test_stressor_deadline_fires_without_stop(ctx, dev):
    """The host never raises the flag before the deadline: every work-group
    exits on its own deadline and the report says so."""
    import time
    w = synth.u32(5, 4096)
    st = ctx.stressor("vl1d", 0.125, src0=_t(w.view(np.int32), dev), n=4096, deadline_ms=30)
    time.sleep(0.2)
    rep = st.stop(raise_on_timeout=False)
    assert rep.timed_out and rep.status == 4
    rec = st.records()
    assert np.all(rec["flags"] & 1)
    exp = oracle.cache_wg_expected(w, rec["work"])
    assert np.array_equal(rec["check"].astype(np.uint32), exp)


def test_invalid_arguments_rejected(ctx, dev):
    from paper_2501_16909_amd import coloc
    w = _t(synth.u32(5, 4096).view(np.int32), dev)
    for bad in (dict(resource="hbm", x=0.5),                        # missing operands
                dict(resource="l2", x=0.5, src0=w, n=1000),         # span not a multiple
                dict(resource="valu_f32", x=0.5, dst=w, knob=3),    # bad ILP
                dict(resource="lds", x=0.5, src0=w, vec=3)):
        r, x = bad.pop("resource"), bad.pop("x")
        with pytest.raises(coloc.CiError) as ei:
            ctx.stressor(r, x, **bad)
        assert ei.value.status == 1
    with pytest.raises(coloc.CiError):
        ctx.stressor("hbm", 1.5)
    with pytest.raises(coloc.CiError):
        ctx.stressor("hbm", float("nan"))
    # a zero-intensity stressor is a valid no-op
    rep = ctx.stressor("hbm", 0.0).stop()
    assert rep.grid == 0 and rep.ncu == 0


# ------------------------------------------------------------ VALU FP64
@pytest.mark.parametrize("ilp,iters,passes,x,a", [(1, 4096, 1, 0.125, 1 - 2.0 ** -20),
                                                  (4, 1000, 3, 0.5, 1 + 2.0 ** -20),
                                                  (8, 13, 2, 1 / 32, 0.5), (2, 100, 1, 1.0, 2.0)])
def test_valu64_stressor_fixed(ctx, dev, ilp, iters, passes, x, a):
    import torch
    ncu = 8 * round(32 * x)
    threads = ncu * 4 * 256
    out = torch.empty(threads * ilp, dtype=torch.float64, device=dev)
    st = ctx.stressor("valu_f64", x, dst=out, knob=ilp, iters=iters, passes=passes, fa=a)
    rep = st.stop()
    got = out.cpu().numpy().reshape(threads, ilp)
    sel = np.unique(np.concatenate([np.arange(0, threads, 89), [threads - 1]]))
    want = oracle.valu64_outputs(sel, ilp, a, iters * passes)
    assert np.array_equal(got[sel].view(np.uint64), want.view(np.uint64))
    assert rep.units == float(threads) * ilp * iters * passes


# ------------------------------------------------------------ duty cycle
def test_duty_cycle_keeps_results_and_scales_time(ctx, dev):
    """A duty-cycled stressor does the same work with the same results; it
    only idles between stretches of work.  With one wave per SIMD nothing
    else fills the idle issue slots, so at a fixed clock the launch takes
    100/duty times as long; with several waves per SIMD the rate still falls
    with duty."""
    import torch
    a, b = 1 - 2.0 ** -12, 2.0 ** -12

    def run(duty, wg, iters, passes):
        threads = 256 * wg * 256
        out = torch.empty(threads * 4, dtype=torch.float32, device=dev)
        rep = ctx.stressor("valu_f32", 1.0, dst=out, knob=4, iters=iters, passes=passes, fa=a, fb=b,
                           wg_per_cu=wg, threads=256, duty=duty).stop()
        assert rep.units == 2.0 * threads * 4 * iters * passes
        return out.cpu().numpy(), rep.kernel_ns

    outs, times = {}, {}
    for duty in (100, 50, 25):
        outs[duty], times[duty] = run(duty, 1, 40000, 8)
    assert np.array_equal(outs[100].view(np.uint32), outs[50].view(np.uint32))
    assert np.array_equal(outs[100].view(np.uint32), outs[25].view(np.uint32))
    threads = 256 * 256
    sel = np.arange(0, threads, 1013)
    want = oracle.valu_outputs(sel, 4, a, b, 40000 * 8)
    assert np.array_equal(outs[25].reshape(threads, 4)[sel].view(np.uint32), want.view(np.uint32))
    # the wave idles as long as it worked at 50% and three times as long at
    # 25%: twice the launch time.  Against 100% the ratio is smaller: with the
    # VALUs of every CU busy the chip lowers its clock, at half duty it does not.
    assert 1.8 < times[25] / times[50] < 2.2, times
    assert 1.15 < times[50] / times[100] < 2.2, times
    # default shape: four work-groups per CU share each SIMD
    t4 = {d: run(d, 4, 20000, 4)[1] for d in (100, 50, 25)}
    assert t4[100] < t4[50] < t4[25], t4
    # the MFMA and LDS loops keep their results under a duty cycle too
    da, db, fa, fb = _mfma_operands("bf16", "ones")
    waves = 256 * 2 * 4
    out = torch.empty(waves * 4 * 1024, dtype=torch.float32, device=dev)
    ctx.stressor("mfma_bf16", 1.0, src0=_t(da, dev), src1=_t(db, dev), dst=out, knob=4, iters=100,
                 passes=3, duty=40).stop()
    assert np.all(out.cpu().numpy().reshape(-1, 32, 32) == oracle.mfma_tile_expected(fa, fb, 300))
    w = synth.u32(synth.seed_for(1, synth.BUF_LDS), 8192)
    for vec in (1, 4):
        st = ctx.stressor("lds", 0.25, src0=_t(w.view(np.int32), dev), vec=vec, knob=3, passes=3, duty=30)
        st.stop()
        rec = st.records()
        assert np.array_equal(rec["check"].astype(np.uint32),
                              oracle.lds_wg_expected(w, vec, 3, waves=16, passes=rec["work"]))


def test_duty_out_of_range_rejected(ctx, dev):
    from paper_2501_16909_amd import coloc
    import torch
    out = torch.empty(1 << 16, dtype=torch.float32, device=dev)
    with pytest.raises(coloc.CiError) as ei:
        ctx.stressor("valu_f32", 0.25, dst=out, duty=101)
    assert ei.value.status == 1
