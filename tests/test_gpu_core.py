"""GPU parity of the core path: placement under CU masks, the device input
fill, the triad victim, the HBM (triad) stressor, colocation and the
zero-intensity invariant.  Every comparison is against the CPU oracle."""
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


def test_device_info(ctx):
    info = ctx.info
    assert info.num_cus == 256, info.num_cus
    assert info.arch.decode().startswith("gfx950")
    assert info.wave_size == 64
    assert info.wall_clock_khz > 0
    assert ctx.peak("hbm") == 8.0e12


def test_placement_full_and_single_bits(ctx):
    locs = ctx.probe_placement(None, 8192)
    xcc = (locs >> 8) & 0xF
    assert set(xcc.tolist()) == set(range(8))
    assert len(set(locs.tolist())) == 256
    # eight consecutive CU-mask bits 8j..8j+7 select one CU on every XCD:
    # bit b lands on XCD b mod 8
    seen = set()
    for j in (0, 1, 5, 31):
        mask = [0] * 8
        for b in range(8 * j, 8 * j + 8):
            mask[b // 32] |= 1 << (b % 32)
        l = ctx.probe_placement(mask, 512)
        cus = set(l.tolist())
        assert len(cus) == 8, (j, sorted(cus))
        assert sorted((c >> 8) & 0xF for c in cus) == list(range(8))
        assert not (cus & seen)
        seen |= cus
    # a mask that leaves an XCD without CUs is refused
    from paper_2501_16909_amd import coloc
    with pytest.raises(coloc.CiError) as ei:
        ctx.probe_placement([1, 0, 0, 0, 0, 0, 0, 0], 64)
    assert ei.value.status == 1


@pytest.mark.parametrize("x", [1 / 32, 0.25, 0.5, 0.75, 0.3])
def test_intensity_masks_are_balanced(ctx, x):
    mask, ncu = ctx.cu_mask(x)
    assert ncu == 8 * round(32 * x)
    l = ctx.probe_placement(mask, 16384)
    cus = set(l.tolist())
    assert len(cus) == ncu
    per_xcd = np.bincount([(c >> 8) & 0xF for c in cus], minlength=8)
    assert per_xcd.max() == per_xcd.min() == ncu // 8
    comp, nc = ctx.cu_mask(x, complement=True)
    lc = set(ctx.probe_placement(comp, 16384).tolist())
    assert len(lc) == nc and not (lc & cus)
    # within each XCD the CUs spread over its shader engines as evenly as
    # the count allows, for the mask and its complement alike
    for sel in (cus, lc):
        per_se = np.bincount([((c >> 8) & 0xF) * 4 + ((c >> 5) & 3) for c in sel], minlength=32)
        assert per_se.max() - per_se.min() <= 1, per_se


def test_device_fill_matches_host_generator(ctx, dev):
    import torch
    n = (1 << 20) + 77
    t = torch.empty(n, dtype=torch.float32, device=dev)
    synth.device_fill_uniform_f32(t.data_ptr(), n, 12345, start=5)
    torch.cuda.synchronize()
    assert np.array_equal(t.cpu().numpy().view(np.uint32),
                          synth.uniform_f32(12345, n, start=5).view(np.uint32))
    w = torch.empty(n, dtype=torch.int32, device=dev)
    synth.device_fill_u32(w.data_ptr(), n, 999)
    torch.cuda.synchronize()
    assert np.array_equal(w.cpu().numpy().view(np.uint32), synth.u32(999, n))


@pytest.mark.parametrize("n,passes,in_kernel", [(0, 1, False), (1, 1, False), (1023, 1, False), (1024, 2, False),
                                                ((1 << 20) + 333, 3, False), (1 << 22, 1, False),
                                                (1023, 3, True), ((1 << 20) + 333, 5, True), (1 << 22, 2, True)])
def test_triad_victim_matches_oracle(ctx, dev, n, passes, in_kernel):
    import torch
    b = synth.uniform_f32(synth.seed_for(0, synth.BUF_B), n)
    c = synth.uniform_f32(synth.seed_for(0, synth.BUF_C), n)
    tb, tc = _t(b, dev), _t(c, dev)
    ta = torch.full((max(n, 1),), float("nan"), device=dev)[:n]
    r = ctx.victim_triad(tb, tc, ta, passes=passes, in_kernel=in_kernel)
    want = oracle.triad_f32(b, c)
    got = ta.cpu().numpy()
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    assert r.checksum_bits == oracle.bitsum_u32(want)
    assert oracle.rel_err_sum(r.sum_f64, want) <= 1e-6
    assert r.time_ns > 0 or n == 0
    assert r.t_end >= r.t_begin


def test_victim_flags_validated(ctx, dev):
    import torch
    from paper_2501_16909_amd import coloc
    t = torch.zeros(1024, dtype=torch.float32, device=dev)
    d = ctx.triad_desc(t, t, t, passes=1)
    d.flags = 2
    with pytest.raises(coloc.CiError) as ei:
        ctx.victim_run(d)
    assert ei.value.status == 1
    d.flags, d.reserved = 0, 1
    with pytest.raises(coloc.CiError) as ei:
        ctx.victim_run(d)
    assert ei.value.status == 1


def test_triad_sum_relative_error_full_size(ctx, dev):
    """N = 2^30 (4 GiB per array): outputs checked on sampled indices
    regenerated from the counter-form generator; the FP64 checksum against
    the closed-form identity sum a ~ sum b + 3 sum c."""
    import torch
    n = 1 << 30
    sb, sc = synth.seed_for(1, synth.BUF_B), synth.seed_for(1, synth.BUF_C)
    tb = torch.empty(n, dtype=torch.float32, device=dev)
    tc = torch.empty(n, dtype=torch.float32, device=dev)
    synth.device_fill_uniform_f32(tb.data_ptr(), n, sb)
    synth.device_fill_uniform_f32(tc.data_ptr(), n, sc)
    torch.cuda.synchronize()
    ta = torch.empty_like(tb)
    r = ctx.victim_triad(tb, tc, ta, passes=1)
    idx = np.unique(np.concatenate([np.arange(64), n - 1 - np.arange(64),
                                    (synth.words(77, 4096) % np.uint64(n)).astype(np.int64)]))
    want = oracle.triad_f32(synth.uniform_f32_at(sb, idx), synth.uniform_f32_at(sc, idx))
    got = ta[torch.from_numpy(idx).to(dev)].cpu().numpy()
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    # device sums of the inputs and the output obey the triad identity
    bits_b, sum_b = ctx.checksum(tb)
    bits_c, sum_c = ctx.checksum(tc)
    absum = float((3 * tc.abs().double().sum() + ta.abs().double().sum()).item())
    assert abs(r.sum_f64 - (sum_b + 3 * sum_c)) <= 2.0 ** -24 * absum * 1.01 + 1e-6 * abs(r.sum_f64)
    del tb, tc, ta
    torch.cuda.empty_cache()


def _hbm_buffers(dev, n, cfg=0):
    b = synth.uniform_f32(synth.seed_for(cfg, synth.BUF_B2), n)
    c = synth.uniform_f32(synth.seed_for(cfg, synth.BUF_C2), n)
    import torch
    return b, c, _t(b, dev), _t(c, dev), torch.empty(n, dtype=torch.float32, device=dev)


@pytest.mark.parametrize("x,passes,n", [(1.0, 1, (1 << 22) + 5), (0.5, 3, 1 << 20), (1 / 32, 2, 5000)])
def test_hbm_stressor_fixed_passes(ctx, dev, x, passes, n):
    b, c, tb, tc, ta = _hbm_buffers(dev, n)
    st = ctx.stressor("hbm", x, src0=tb, src1=tc, dst=ta, n=n, passes=passes)
    rep = st.stop()
    want = oracle.triad_f32(b, c)
    assert np.array_equal(ta.cpu().numpy().view(np.uint32), want.view(np.uint32))
    ncu = 8 * round(32 * x)
    assert rep.grid == ncu and rep.wg_reported == rep.grid
    chunks = (n + 1023) // 1024                   # default wave-chunk: 4 x 16 B per lane
    assert rep.work == passes * chunks
    assert rep.units == 12.0 * n * passes
    assert rep.distinct_cus == ncu


def test_hbm_stressor_triad_full_size_benchmark_shape(ctx, dev):
    """The benchmark's roofline launch itself: the HBM triad over N = 2^30
    (4 GiB per array) at full intensity with default options (256
    work-groups of 512 threads, one pass, fixed work).  Outputs on sampled
    indices against the oracle on inputs regenerated from the counter-form
    generator; every wave-chunk done once; the FP64 sum of the output
    against the triad identity of the input sums."""
    import torch
    n = 1 << 30
    sb, sc = synth.seed_for(1, synth.BUF_B), synth.seed_for(1, synth.BUF_C)
    tb = torch.empty(n, dtype=torch.float32, device=dev)
    tc = torch.empty_like(tb)
    ta = torch.empty_like(tb)
    synth.device_fill_uniform_f32(tb.data_ptr(), n, sb)
    synth.device_fill_uniform_f32(tc.data_ptr(), n, sc)
    torch.cuda.synchronize()
    rep = ctx.stressor("hbm", 1.0, src0=tb, src1=tc, dst=ta, n=n, passes=1).stop()
    assert rep.grid == 256 and rep.wg_reported == 256 and not rep.timed_out
    assert rep.work == n // 1024 and rep.units == 12.0 * n
    idx = np.unique(np.concatenate([np.arange(64), n - 1 - np.arange(64),
                                    (synth.words(91, 4096) % np.uint64(n)).astype(np.int64)]))
    want = oracle.triad_f32(synth.uniform_f32_at(sb, idx), synth.uniform_f32_at(sc, idx))
    got = ta[torch.from_numpy(idx).to(dev)].cpu().numpy()
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    _, sum_a = ctx.checksum(ta)
    _, sum_b = ctx.checksum(tb)
    _, sum_c = ctx.checksum(tc)
    absum = float((3 * tc.abs().double().sum() + ta.abs().double().sum()).item())
    assert abs(sum_a - (sum_b + 3 * sum_c)) <= 2.0 ** -24 * absum * 1.01 + 1e-6 * abs(sum_a)
    print(f"hbm triad 2^30: {rep.achieved / 1e9:.0f} GB/s ({rep.pct_of_peak:.1f} % of peak)")
    del tb, tc, ta
    torch.cuda.empty_cache()


def test_hbm_stressor_persistent_colocated(ctx, dev):
    n_v = 1 << 22
    b = synth.uniform_f32(synth.seed_for(0, synth.BUF_B), n_v)
    c = synth.uniform_f32(synth.seed_for(0, synth.BUF_C), n_v)
    tb, tc = _t(b, dev), _t(c, dev)
    import torch
    ta = torch.empty_like(tb)
    alone = ctx.victim_triad(tb, tc, ta, passes=20)
    sb, sc, tsb, tsc, tsa = _hbm_buffers(dev, 1 << 24)
    with ctx.stressor("hbm", 1.0, src0=tsb, src1=tsc, dst=tsa, n=1 << 24) as st:
        col = ctx.victim_triad(tb, tc, ta, passes=20)
    rep = st.report
    assert not rep.timed_out
    assert col.checksum_bits == alone.checksum_bits
    assert rep.wg_reported == rep.grid
    assert rep.t_last_start <= col.t_begin and rep.t_first_end >= col.t_end, "stressor window"
    assert col.time_ns > 1.05 * alone.time_ns, (alone.time_ns, col.time_ns)
    want = oracle.triad_f32(sb, sc)
    assert np.array_equal(tsa.cpu().numpy().view(np.uint32), want.view(np.uint32))
    print(f"triad alone {alone.time_ns/1e3:.1f} us colocated {col.time_ns/1e3:.1f} us; "
          f"stressor {rep.achieved/1e9:.0f} GB/s")


@pytest.mark.parametrize("mix", ["read", "copy", "write"])
@pytest.mark.parametrize("x,passes,n,vec,chunk", [(1.0, 1, (1 << 22) + 5, 0, 2), (0.5, 3, 1 << 20, 1, 1),
                                                 (1 / 32, 2, 5000, 0, 4), (0.25, 1, 333, 1, 2)])
def test_hbm_mixes_fixed_passes(ctx, dev, mix, x, passes, n, vec, chunk):
    """Read-only, copy and write-only mixes: outputs bit-exact, the read
    checksum mod 2^32 exact, and nothing stored where the mix stores nothing."""
    import torch
    from paper_2501_16909_amd import coloc
    b, c, tb, tc, _ = _hbm_buffers(dev, n, cfg=3)
    sentinel = np.full(n, 0x7FC0DEAD, np.uint32)
    ta = _t(sentinel.view(np.float32), dev)
    ops = {"read": dict(src0=tb, src1=tc), "copy": dict(src0=tb, dst=ta), "write": dict(dst=ta)}[mix]
    rep = ctx.stressor("hbm", x, n=n, passes=passes, vec=vec, chunk=chunk, knob=coloc.HBM_MIX[mix],
                       **ops).stop()
    got = ta.cpu().numpy().view(np.uint32)
    if mix == "read":
        assert np.array_equal(got, sentinel)
        assert rep.checksum % 2 ** 32 == oracle.hbm_read_checksum(b, c, passes)
    elif mix == "copy":
        assert np.array_equal(got, oracle.hbm_copy(b))
    else:
        assert np.array_equal(got, oracle.hbm_write_pattern(n))
    ncu = 8 * round(32 * x)
    assert rep.grid == ncu and rep.wg_reported == rep.grid and not rep.timed_out
    assert rep.work == passes * ((n + 256 * chunk - 1) // (256 * chunk))
    assert rep.units == oracle.hbm_bytes_per_element(mix) * n * passes
    # the inputs are left as they were
    assert np.array_equal(tb.cpu().numpy().view(np.uint32), b.view(np.uint32))


def test_hbm_mix_options_are_checked(ctx, dev):
    import torch
    from paper_2501_16909_amd import coloc
    t = torch.empty(1024, dtype=torch.float32, device=dev)
    for bad in (dict(knob=5, src0=t, src1=t, dst=t), dict(knob=coloc.HBM_MIX["read"], src0=t),
                dict(knob=coloc.HBM_MIX["copy"], src0=t), dict(knob=coloc.HBM_MIX["write"]),
                dict(knob=coloc.HBM_MIX["copy"], src0=t[1:], dst=t),
                dict(src0=t, src1=t, dst=t, chunk=3)):
        with pytest.raises(coloc.CiError) as ei:
            ctx.stressor("hbm", 0.25, n=512, passes=1, **bad)
        assert ei.value.status == 1, bad


def test_hbm_read_mix_full_size_closed_form(ctx, dev):
    """N = 2^30 words per array: b holds the words 0..N-1 and c zeros, so the
    read checksum is passes * N(N-1)/2 mod 2^32; the persistent form reports
    8 bytes per element of every chunk it read."""
    import torch
    from paper_2501_16909_amd import coloc
    n = 1 << 30
    tb = torch.arange(n, dtype=torch.int32, device=dev).view(torch.float32)
    tc = torch.zeros(n, dtype=torch.float32, device=dev)
    rep = ctx.stressor("hbm", 1.0, src0=tb, src1=tc, n=n, passes=2, knob=coloc.HBM_MIX["read"]).stop()
    assert rep.checksum % 2 ** 32 == (2 * (n * (n - 1) // 2)) % 2 ** 32
    assert rep.units == 16.0 * n and rep.wg_reported == rep.grid
    import time
    with ctx.stressor("hbm", 1.0, src0=tb, src1=tc, n=n, knob=coloc.HBM_MIX["read"]) as st:
        time.sleep(0.02)
    r = st.report
    assert not r.timed_out and r.wg_reported == r.grid
    assert r.units == 8.0 * 1024 * r.work and r.work > 0
    print(f"read mix: fixed {rep.achieved / 1e9:.0f} GB/s ({rep.pct_of_peak:.1f} %), "
          f"persistent {r.achieved / 1e9:.0f} GB/s")
    del tb, tc
    torch.cuda.empty_cache()


def test_hbm_mixes_colocated(ctx, dev):
    """Persistent read-only and write-only mixes beside a triad victim: every
    colocated run inside the stressor window, outputs equal to the alone
    run, and the stressor's own rate reported per cell."""
    import torch
    from paper_2501_16909_amd import coloc
    n = 1 << 22
    tb = _t(synth.uniform_f32(synth.seed_for(0, synth.BUF_B), n), dev)
    tc = _t(synth.uniform_f32(synth.seed_for(0, synth.BUF_C), n), dev)
    ta = torch.empty_like(tb)
    d = ctx.triad_desc(tb, tc, ta, passes=8)
    m = 1 << 26
    sb, sc, sa = (torch.empty(m, dtype=torch.float32, device=dev) for _ in range(3))
    synth.device_fill_uniform_f32(sb.data_ptr(), m, synth.seed_for(4, synth.BUF_B2))
    synth.device_fill_uniform_f32(sc.data_ptr(), m, synth.seed_for(4, synth.BUF_C2))
    torch.cuda.synchronize()
    opts = [dict(src0=sb, src1=sc, n=m, knob=coloc.HBM_MIX["read"]),
            dict(dst=sa, n=m, knob=coloc.HBM_MIX["write"])]
    cells = ctx.measure_sensitivity(d, ["hbm", "hbm"], opts, [0.5], reps=8, warmups=2)
    for cell in cells:
        assert cell["output_equal"] and cell["window_covered"] and not cell["timed_out"], cell
        assert cell["stressor_achieved"] > 1e12 and cell["slowdown"] > 1.02, cell
    print("read / write mix at 0.5:", [round(c["slowdown"], 3) for c in cells])


def test_zero_intensity_invariant(ctx, dev):
    """A stressor at intensity 0 launches nothing: slowdown 1.00 +- 0.02."""
    import torch
    n = 1 << 22
    b = synth.uniform_f32(synth.seed_for(0, synth.BUF_B), n)
    c = synth.uniform_f32(synth.seed_for(0, synth.BUF_C), n)
    tb, tc = _t(b, dev), _t(c, dev)
    ta = torch.empty_like(tb)
    _, _, tsb, tsc, tsa = _hbm_buffers(dev, 1 << 22)
    # a victim of about 0.1 ms, warm-up for the clock to settle after whatever
    # ran before, and enough counterbalanced pairs for a stable median;
    # run-to-run jitter of single runs is a few percent
    d = ctx.triad_desc(tb, tc, ta, passes=40)
    cells = ctx.measure_sensitivity(d, ["hbm"], [dict(src0=tsb, src1=tsc, dst=tsa, n=1 << 22)], [0.0, 1.0],
                                    reps=41, warmups=20)
    z, full = cells
    assert abs(z["slowdown"] - 1.0) <= 0.02, z
    # bootstrap interval of each cell: ordered, and at zero intensity it
    # reaches 1.00 within the invariant's tolerance
    for cell in cells:
        assert cell["slowdown_ci_lo"] <= cell["slowdown_ci_hi"], cell
    assert z["slowdown_ci_lo"] <= 1.02 and z["slowdown_ci_hi"] >= 0.98, z
    assert z["output_equal"] and full["output_equal"]
    assert full["window_covered"], full
    assert full["slowdown"] > 1.1, full
    print("cells:", cells)


def test_disjoint_idle_stressor_costs_nothing(ctx, dev):
    """A sleeping occupancy hog on CUs the victim does not use takes nothing
    the victim needs: with the queue-pair check in place the victim keeps its
    alone speed on the complement CUs (1.00 +- 0.06 for a short victim).
    The victim is one launch (one sweep of 384 MiB): a victim of many short
    launches also pays the command processor's time between its launches,
    which grows when another queue is active."""
    import torch
    n = 1 << 25
    tb = _t(synth.uniform_f32(synth.seed_for(0, synth.BUF_B), n), dev)
    tc = _t(synth.uniform_f32(synth.seed_for(0, synth.BUF_C), n), dev)
    ta = torch.empty_like(tb)
    d = ctx.triad_desc(tb, tc, ta, passes=1)
    cells = ctx.measure_sensitivity(d, ["occupancy"], [dict()], [0.25, 0.5], reps=16, warmups=3,
                                    placement="disjoint")
    for c in cells:
        assert c["output_equal"] and c["window_covered"], c
        info = {k: c[k] for k in ("intensity", "slowdown", "slowdown_ci_lo", "slowdown_ci_hi", "t_alone_ns",
                                  "t_col_ns", "queue_unresolved")}
        assert abs(c["slowdown"] - 1.0) <= 0.06, info
    st = ctx.queue_stats()
    assert st["checks"] >= 1, st
    print("queue-pair check:", st, [round(c["slowdown"], 3) for c in cells])


def test_disjoint_sweep_of_many_intensities_keeps_its_victim_stream(ctx, dev):
    """Six intensities on disjoint CUs need more CU-masked queues than the
    stream cache keeps (the victim's complement masks and the stressor's
    masks): the cache must never drop the victim stream a cell is measuring
    on.  Every cell is measured, finite, covered and output-equal, and the
    per-rep times come back for every rep."""
    import torch
    n = 1 << 22
    tb = _t(synth.uniform_f32(synth.seed_for(0, synth.BUF_B), n), dev)
    tc = _t(synth.uniform_f32(synth.seed_for(0, synth.BUF_C), n), dev)
    ta = torch.empty_like(tb)
    _, _, tsb, tsc, tsa = _hbm_buffers(dev, 1 << 22)
    d = ctx.triad_desc(tb, tc, ta, passes=4)
    xs = [0.125, 0.25, 0.375, 0.5, 0.625, 0.75]
    cells = ctx.measure_sensitivity(d, ["hbm"], [dict(src0=tsb, src1=tsc, dst=tsa, n=1 << 22)], xs, reps=4,
                                    warmups=1, placement="disjoint")
    assert [c["intensity"] for c in cells] == xs
    for c in cells:
        assert np.isfinite(c["slowdown"]) and c["slowdown"] > 0.5, c
        assert c["output_equal"] and c["window_covered"], c
        assert len(c["rep_alone_ns"]) == 4 and all(np.isfinite(c["rep_alone_ns"])), c
        assert all(np.isfinite(c["rep_col_ns"])), c
        # the cell's median slowdown is the ratio of the per-rep medians
        assert c["slowdown"] == pytest.approx(np.median(c["rep_col_ns"]) / np.median(c["rep_alone_ns"]), rel=1e-12)
    print("disjoint sweep:", [round(c["slowdown"], 3) for c in cells], ctx.queue_stats())


def test_stamps_bracket_enqueued_work(ctx, dev):
    """ci_stamp writes the device clock that victim_run's stamps use: two
    stamps around enqueued work are ordered and precede a later victim."""
    import torch
    n = 1 << 22
    tb = _t(synth.uniform_f32(synth.seed_for(0, synth.BUF_B), n), dev)
    tc = _t(synth.uniform_f32(synth.seed_for(0, synth.BUF_C), n), dev)
    ta = torch.empty_like(tb)
    d = ctx.triad_desc(tb, tc, ta, passes=4)
    side = torch.cuda.Stream(device=dev)
    slots = torch.zeros(2, dtype=torch.int64, device=dev)
    ctx.stamp(slots[0:1], side)
    ctx.victim_enqueue(d, side, 8)
    ctx.stamp(slots[1:2], side)
    side.synchronize()
    s0, s1 = (int(v) for v in slots.cpu().tolist())
    assert 0 < s0 < s1
    # 8 launches of 4 passes over 48 MiB take well over 10 us
    ticks_us = ctx.info.wall_clock_khz / 1e3
    assert (s1 - s0) / ticks_us > 10.0
    out = ctx.victim_run(d)
    assert out.t_begin > s1 and out.t_end > out.t_begin
    from paper_2501_16909_amd import coloc
    with pytest.raises(coloc.CiError):
        ctx.stamp(slots[0:1], None)


def test_raw_placement_flag_skips_the_queue_check(ctx, dev):
    import torch
    n = 1 << 22
    tb = _t(synth.uniform_f32(synth.seed_for(0, synth.BUF_B), n), dev)
    tc = _t(synth.uniform_f32(synth.seed_for(0, synth.BUF_C), n), dev)
    ta = torch.empty_like(tb)
    d = ctx.triad_desc(tb, tc, ta, passes=4)
    before = ctx.queue_stats()["checks"]
    cell, = ctx.measure_sensitivity(d, ["occupancy"], [dict()], [0.5], reps=4, warmups=1,
                                    placement="disjoint", queue_check=False)
    assert cell["output_equal"] and cell["window_covered"] and cell["reps"] == 4
    assert ctx.queue_stats()["checks"] == before
    cell, = ctx.measure_sensitivity(d, ["occupancy"], [dict()], [0.5], reps=4, warmups=1,
                                    placement="disjoint")
    assert ctx.queue_stats()["checks"] == before + 1
