"""GPU tests of the continuous-batching colocation loop (serve_run):
requests arriving while others run are admitted as memory and slots free
up, overlap on the device, and each result equals the same request served
alone and the oracle's result on regenerated inputs."""
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


def _trace():
    reqs = []
    t = 0.0
    sizes = [("triad", dict(n=(1 << 20) + 7)), ("gemm", dict(m=256, n=384, k=512, dtype="bf16")),
             ("gemv", dict(n=1024, k=2048, dtype="bf16")), ("triad", dict(n=1 << 22)),
             ("gemm", dict(m=512, n=512, k=1024, dtype="bf16")), ("gemv", dict(n=4096, k=4096, dtype="bf16")),
             ("gemm", dict(m=1024, n=1024, k=1024, dtype="f32")), ("triad", dict(n=3 << 20)),
             ("gemv", dict(n=333, k=4104, dtype="bf16")), ("gemm", dict(m=130, n=70, k=64, dtype="bf16"))]
    for i, (kind, kw) in enumerate(sizes * 2):
        q = {"arrival_s": t, "kind": kind, "seed": 5000 + 10 * i}
        q.update(kw)
        reqs.append(q)
        t += 0.0007 * (1 + (i % 3))
    return reqs


def _oracle_check(q, served, got=None):
    """The served result against the oracle on regenerated inputs: the
    loop's checksums, and, when the output copy `got` is given, every
    element (triad bit for bit, GEMM and GEMV within the accumulation
    bound of each entry)."""
    s = q["seed"]
    if q["kind"] == "triad":
        b = synth.uniform_f32(s, q["n"])
        c = synth.uniform_f32(s + 1, q["n"])
        want = oracle.triad_f32(b, c)
        assert served["checksum_bits"] == oracle.bitsum_u32(want)
        if got is not None:
            assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), q
        return
    if q["kind"] == "gemm":
        m, n, k = q["m"], q["n"], q["k"]
        a = synth.uniform_f32(s, m * k).reshape(m, k)
        b = synth.uniform_f32(s + 1, n * k).reshape(n, k)
        if q["dtype"] == "bf16":
            fa, fb = oracle.bf16_to_f64(oracle.f32_to_bf16(a)), oracle.bf16_to_f64(oracle.f32_to_bf16(b))
        else:
            fa, fb = a.astype(np.float64), b.astype(np.float64)
        want = oracle.gemm_f64(fa, fb)
        bound = oracle.accumulation_bound(k + 1, oracle.gemm_abs_f64(fa, fb), 2.0 ** -23)
    else:
        n, k = q["n"], q["k"]
        w = oracle.bf16_to_f64(oracle.f32_to_bf16(synth.uniform_f32(s, n * k))).reshape(n, k)
        x = oracle.bf16_to_f64(oracle.f32_to_bf16(synth.uniform_f32(s + 1, k)))
        want = oracle.gemv_f64(w, x)
        bound = oracle.accumulation_bound(k + 1, np.abs(w) @ np.abs(x), 2.0 ** -23)
    # the loop reports the FP64 sum of the FP32 outputs: within the summed bound
    # plus the FP64 rounding of that sum
    tol = float(np.sum(bound)) + 1e-12 * float(np.sum(np.abs(want))) * want.size
    assert abs(served["sum_f64"] - float(np.sum(want))) <= tol, (q, served["sum_f64"], float(np.sum(want)))
    if got is not None:
        got = got.astype(np.float64).reshape(want.shape)
        assert np.all(np.abs(got - want) <= bound), (q, float(np.max(np.abs(got - want) / np.maximum(bound, 1e-300))))
        assert oracle.bitsum_u32(got.astype(np.float32)) == served["checksum_bits"]


def _with_copies(reqs, dev):
    import torch
    for q in reqs:
        n = q["m"] * q["n"] if q["kind"] == "gemm" else q["n"]
        q["out_copy"] = torch.full((n,), float("nan"), dtype=torch.float32, device=dev)
    return reqs


def test_serve_naive_overlaps_and_matches_isolated(ctx, dev):
    reqs = _with_copies(_trace(), dev)
    out = ctx.serve(reqs, policy="naive", hbm_budget=1 << 30, slots=4)
    assert all(o["status"] == 0 for o in out)
    for q, o in zip(reqs, out):
        assert o["admit_s"] >= q["arrival_s"] - 1e-9 and o["end_s"] > o["admit_s"]
        assert 0 <= o["slot"] < 4 and o["service_ns"] > 0
    # requests that arrive together run together: four are admitted before
    # the first completion is observed
    burst = ctx.serve([dict(r, arrival_s=0.0) for r in reqs], policy="naive", hbm_budget=1 << 30, slots=4)
    spans = sorted((o["admit_s"], o["end_s"]) for o in burst)
    assert any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))
    assert [o["checksum_bits"] for o in burst] == [o["checksum_bits"] for o in out]
    # same result alone and in the mix (bit for bit, element by element), and
    # every element against the oracle
    import torch
    for q, o in zip(reqs, out):
        mixed = q["out_copy"].cpu().numpy()
        alone_copy = torch.full_like(q["out_copy"], float("nan"))
        alone = ctx.serve([dict(q, arrival_s=0.0, out_copy=alone_copy)], policy="naive", hbm_budget=1 << 30,
                          slots=1)[0]
        assert alone["checksum_bits"] == o["checksum_bits"], q
        assert np.array_equal(alone_copy.cpu().numpy().view(np.uint32), mixed.view(np.uint32)), q
        _oracle_check(q, o, mixed)


def test_serve_budget_and_slots_bound_concurrency(ctx):
    reqs = [dict(r, arrival_s=0.0) for r in _trace()]
    out = ctx.serve(reqs, policy="naive", hbm_budget=128 << 20, slots=2)
    assert all(o["status"] == 0 for o in out)
    ev = sorted([(o["admit_s"], 1) for o in out] + [(o["end_s"], -1) for o in out])
    live = peak = 0
    for _, d in ev:
        live += d
        peak = max(peak, live)
    assert peak <= 2
    # FIFO without bypass: admission order is arrival (index) order
    order = [i for i, _ in sorted(enumerate(out), key=lambda kv: kv[1]["admit_s"])]
    assert order == sorted(order)


def test_serve_sensitivity_policy_serialises_fragile_mix(ctx):
    """Profiles that predict a large slowdown for any pair: the sensitivity
    policy runs requests one at a time; with an unbounded bound it behaves
    like the naive policy."""
    fragile = {"sens": {"hbm": [1.0, 2.0, 3.0, 4.0, 5.0]}, "press": {"hbm": 0.6}, "occ": 0.3}
    profiles = {"triad": fragile, "gemm": fragile, "gemv": fragile}
    reqs = [dict(r, arrival_s=0.0) for r in _trace()[:8]]
    out = ctx.serve(reqs, policy="sensitivity", bound=1.5, hbm_budget=1 << 30, slots=4,
                    profiles=profiles)
    spans = sorted((o["admit_s"], o["end_s"]) for o in out)
    assert all(spans[i + 1][0] >= spans[i][1] - 1e-6 for i in range(len(spans) - 1))
    out2 = ctx.serve(reqs, policy="sensitivity", bound=float("inf"), hbm_budget=1 << 30, slots=4,
                     profiles=profiles)
    spans2 = sorted((o["admit_s"], o["end_s"]) for o in out2)
    assert any(spans2[i + 1][0] < spans2[i][1] for i in range(len(spans2) - 1))
    for a, b in zip(out, out2):
        assert a["checksum_bits"] == b["checksum_bits"]


def _replay_job(p):
    # the library stores curves and pressures as FP32: the oracle sees the
    # same rounded values
    from paper_2501_16909_amd import coloc
    f32 = lambda v: float(np.float32(v))
    job = {"sens": [[f32(v) for v in p["sens"].get(r, [1.0] * 5)] for r in coloc.RESOURCES],
           "press": [f32(p["press"].get(r, 0.0)) for r in coloc.RESOURCES],
           "bytes": 1, "occ": f32(p["occ"]), "hbm_write_frac": f32(p.get("hbm_write_frac", 1.0)),
           "press_hbm_read": f32(p.get("press_hbm_read", 0.0))}
    if "sens_hbm_read" in p:
        job["sens_hbm_read"] = [f32(v) for v in p["sens_hbm_read"]]
    return job


@pytest.mark.parametrize("read_curves", [False, True])
def test_serve_admissions_replay_against_oracle(ctx, read_curves):
    """Discrete-event replay of the loop's own log: given the completion
    order the loop observed, every admission is one the oracle's admission
    rule allows, and no request waited through a completion after which the
    rule would already have allowed it (FIFO, no bypass).  With read-only
    HBM curves the read-mostly GEMV is priced on them (ci_predict_slowdown)."""
    profiles = {"gemv": {"sens": {"hbm": [1.0, 1.5, 2.0, 2.5, 3.0]}, "press": {"hbm": 0.2}, "occ": 0.6,
                         "hbm_write_frac": 0.0, "press_hbm_read": 0.15},
                "triad": {"sens": {"hbm": [1.0, 1.1, 1.2, 1.3, 1.4]}, "press": {"hbm": 1.0}, "occ": 0.6,
                          "hbm_write_frac": 1 / 3, "press_hbm_read": 0.95},
                "gemm": {"sens": {"lds": [1.0] * 5}, "press": {"mfma_bf16": 0.9}, "occ": 0.3,
                         "hbm_write_frac": 0.5}}
    if read_curves:
        profiles["gemv"]["sens_hbm_read"] = [1.0, 1.1, 1.2, 1.3, 1.4]
        profiles["triad"]["sens_hbm_read"] = [1.0, 1.05, 1.1, 1.15, 1.2]
    # requests of 0.1-0.5 ms each, so that completions are spaced out
    sizes = [("gemv", dict(n=16384, k=16384, dtype="bf16")), ("triad", dict(n=1 << 27)),
             ("gemm", dict(m=4096, n=4096, k=4096, dtype="bf16")), ("gemv", dict(n=8192, k=16384, dtype="bf16")),
             ("triad", dict(n=3 << 25)), ("gemm", dict(m=2048, n=4096, k=4096, dtype="bf16"))]
    reqs = []
    for i, (kind, kw) in enumerate(sizes * 3):
        reqs.append(dict(kw, arrival_s=0.0, kind=kind, seed=7000 + 10 * i))
    slots, bound = 3, 1.5
    out = ctx.serve(reqs, policy="sensitivity", bound=bound, hbm_budget=16 << 30, slots=slots,
                    profiles=profiles)
    assert all(o["status"] == 0 for o in out)
    jobs = [_replay_job(profiles[q["kind"]]) for q in reqs]

    def running(t, i):
        return frozenset(j for j, o in enumerate(out) if j != i and o["admit_s"] <= t < o["end_s"])

    order = [i for i, _ in sorted(enumerate(out), key=lambda kv: kv[1]["admit_s"])]
    assert order == sorted(order)                       # FIFO, no bypass
    events = sorted([o["end_s"] for o in out] + [o["admit_s"] for o in out])
    delta = 2e-4   # far longer than one pass of the loop (retire, then admit)
    checked = 0
    for i, o in enumerate(out):
        now = running(o["admit_s"], i)
        assert oracle.admit("sensitivity", [jobs[j] for j in now], jobs[i], 1 << 40, bound, slots), (i, now)
        lo = max(o["arrival_s"], out[i - 1]["admit_s"] if i else 0.0)
        for k, ok in enumerate(out):      # completions while i waited at the front of the queue
            tau = ok["end_s"]
            if not (lo < tau < o["admit_s"]):
                continue
            # only instants after which nothing happened for delta: the loop
            # evaluated exactly this state and left i waiting
            if any(tau < e < tau + delta for e in events):
                continue
            state = running(tau, i)
            assert not oracle.admit("sensitivity", [jobs[j] for j in state], jobs[i], 1 << 40, bound,
                                    slots), (i, k, state)
            checked += 1
    print(f"admissions replayed: {len(out)}, waiting states checked: {checked}")
    # the rule's consequence here: a fragile GEMV never runs beside a triad
    spans = {i: (o["admit_s"], o["end_s"]) for i, o in enumerate(out)}
    for i, qi in enumerate(reqs):
        for j, qj in enumerate(reqs):
            if qi["kind"] == "gemv" and qj["kind"] == "triad":
                a, b = spans[i], spans[j]
                assert a[1] <= b[0] + 1e-9 or b[1] <= a[0] + 1e-9, (i, j)
    starts = sorted(spans.values())
    assert any(starts[i + 1][0] < starts[i][1] for i in range(len(starts) - 1))



def test_serve_under_a_background_stressor(ctx, dev):
    """serve_run_background: an HBM triad stressor on every CU at half duty
    runs for the whole serving run.  Every served result still equals the
    oracle's, the stressor's own output is exact and it drained on its stop
    flag, every admission is one the oracle's rule allows with the
    stressor's load as background, and the rule binds: the fragile GEMV,
    predicted 2x beside the background alone, never overlaps another
    request (without the background it may run beside a GEMM)."""
    import torch
    profiles = {"gemv": {"sens": {"hbm": [1.0, 1.5, 2.0, 2.5, 3.0]}, "press": {"hbm": 0.2}, "occ": 0.6,
                         "hbm_write_frac": 0.0, "press_hbm_read": 0.15},
                "triad": {"sens": {"hbm": [1.0, 1.1, 1.2, 1.3, 1.4]}, "press": {"hbm": 1.0}, "occ": 0.6,
                          "hbm_write_frac": 1 / 3, "press_hbm_read": 0.95},
                "gemm": {"sens": {"lds": [1.0] * 5}, "press": {"mfma_bf16": 0.9}, "occ": 0.3,
                         "hbm_write_frac": 0.5}}
    bg = {"press": {"hbm": 0.5}, "occ": 0.25, "hbm_write_frac": 1 / 3}
    n_s = 1 << 24
    sb = synth.uniform_f32(synth.seed_for(4, synth.BUF_B), n_s)
    sc = synth.uniform_f32(synth.seed_for(4, synth.BUF_C), n_s)
    tsb = torch.from_numpy(np.require(sb, requirements=["C", "W"])).to(dev)
    tsc = torch.from_numpy(np.require(sc, requirements=["C", "W"])).to(dev)
    tsa = torch.empty_like(tsb)
    reqs = _with_copies([dict(q, arrival_s=0.0005 * i) for i, q in enumerate(_trace())], dev)
    slots, bound = 4, 1.6
    print(f"serve_run_background: {len(reqs)} requests, HBM stressor n={n_s} duty 50", flush=True)
    q0 = ctx.queue_stats()
    out, rep = ctx.serve_loaded(reqs, "hbm", 1.0, policy="sensitivity", bound=bound, hbm_budget=1 << 30,
                                slots=slots, profiles=profiles, background=bg, src0=tsb, src1=tsc, dst=tsa,
                                n=n_s, duty=50, deadline_ms=30000)
    assert all(o["status"] == 0 for o in out)
    for q, o in zip(reqs, out):
        _oracle_check(q, o, q["out_copy"].cpu().numpy())
    assert not rep.timed_out and rep.wg_reported == rep.grid and rep.work > 0
    q1 = ctx.queue_stats()
    assert q1["checks"] - q0["checks"] >= slots          # every slot stream checked against its queue
    assert np.array_equal(tsa.cpu().numpy().view(np.uint32), oracle.triad_f32(sb, sc).view(np.uint32))
    jobs = [_replay_job(profiles[q["kind"]]) for q in reqs]
    bgo = _replay_job(dict(bg, sens={}))
    order = [i for i, _ in sorted(enumerate(out), key=lambda kv: kv[1]["admit_s"])]
    assert order == sorted(order)                       # FIFO, no bypass
    for i, o in enumerate(out):
        now = [j for j, oj in enumerate(out) if j != i and oj["admit_s"] <= o["admit_s"] < oj["end_s"]]
        assert oracle.admit("sensitivity", [jobs[j] for j in now], jobs[i], 1 << 40, bound, slots,
                            background=bgo), (i, now)
    spans = [(o["admit_s"], o["end_s"]) for o in out]
    for i, q in enumerate(reqs):
        if q["kind"] != "gemv":
            continue
        for j in range(len(reqs)):
            if j != i:
                assert spans[i][1] <= spans[j][0] + 1e-9 or spans[j][1] <= spans[i][0] + 1e-9, (i, j)
    assert oracle.admit("sensitivity", [jobs[2]], jobs[1], 1 << 40, bound, slots)   # GEMM beside GEMV
    assert not oracle.admit("sensitivity", [jobs[2]], jobs[1], 1 << 40, bound, slots, background=bgo)
    print(f"stressor during serving: {rep.achieved / 1e9:.0f} GB/s over {rep.window_ns / 1e6:.1f} ms")
    # the context is free again: a plain serving run follows
    assert ctx.serve(reqs[:3], policy="naive", hbm_budget=1 << 30, slots=2)[0]["status"] == 0



def test_serve_under_a_background_stressor_occupancy_rule(ctx, dev):
    """The occupancy rule with a background load: requests of occupancy 0.3
    run three at a time on their own (0.9 < 1) but one at a time beside a
    stressor of occupancy 0.5 (0.5 + 0.3 + 0.3 >= 1); every result still
    equals the oracle's."""
    import torch
    prof = {"sens": {"hbm": [1.0] * 5}, "press": {"hbm": 0.1}, "occ": 0.3}
    profiles = {"triad": prof, "gemv": prof, "gemm": prof}
    n_s = 1 << 22
    tsb = torch.zeros(n_s, dtype=torch.float32, device=dev)
    tsc, tsa = torch.zeros_like(tsb), torch.empty_like(tsb)
    reqs = _with_copies([dict(q, arrival_s=0.0) for q in _trace()[:6]], dev)
    print(f"serve_run_background, occupancy rule: {len(reqs)} requests", flush=True)
    out, rep = ctx.serve_loaded(reqs, "hbm", 1.0, policy="usher", hbm_budget=1 << 30, slots=4,
                                profiles=profiles, background={"press": {"hbm": 0.5}, "occ": 0.5},
                                src0=tsb, src1=tsc, dst=tsa, n=n_s, deadline_ms=30000)
    assert all(o["status"] == 0 for o in out) and not rep.timed_out
    for q, o in zip(reqs, out):
        _oracle_check(q, o, q["out_copy"].cpu().numpy())
    spans = sorted((o["admit_s"], o["end_s"]) for o in out)
    assert all(spans[i + 1][0] >= spans[i][1] - 1e-6 for i in range(len(spans) - 1))
    assert np.array_equal(tsa.cpu().numpy(), np.zeros(n_s, np.float32))   # 0 + 3 * 0
    alone = ctx.serve([dict(q) for q in reqs], policy="usher", hbm_budget=1 << 30, slots=4, profiles=profiles)
    spans = sorted((o["admit_s"], o["end_s"]) for o in alone)
    assert any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))


def test_serve_under_a_background_stressor_on_half_the_cus(ctx, dev):
    """A background on half the CUs (the slot check pairs each slot with
    the stressor's own CU mask): every served result equals the oracle's and
    the stressor reports work from exactly half the CUs."""
    import torch
    n_s = 1 << 22
    tsb = torch.zeros(n_s, dtype=torch.float32, device=dev)
    tsc, tsa = torch.zeros_like(tsb), torch.empty_like(tsb)
    reqs = _with_copies([dict(q, arrival_s=0.0002 * i) for i, q in enumerate(_trace()[:6])], dev)
    print(f"serve_run_background at intensity 0.5: {len(reqs)} requests", flush=True)
    q0 = ctx.queue_stats()
    out, rep = ctx.serve_loaded(reqs, "hbm", 0.5, policy="naive", hbm_budget=1 << 30, slots=3,
                                src0=tsb, src1=tsc, dst=tsa, n=n_s, deadline_ms=30000)
    assert all(o["status"] == 0 for o in out) and not rep.timed_out
    for q, o in zip(reqs, out):
        _oracle_check(q, o, q["out_copy"].cpu().numpy())
    assert rep.ncu * 2 == ctx.info.num_cus and rep.distinct_cus == rep.ncu
    assert ctx.queue_stats()["checks"] - q0["checks"] >= 3

def test_serve_under_a_background_stressor_rejects_fixed_passes(ctx, dev):
    import torch
    from paper_2501_16909_amd import coloc
    t = torch.zeros(1 << 16, dtype=torch.float32, device=dev)
    with pytest.raises(coloc.CiError) as ei:
        ctx.serve_loaded(_trace()[:2], "hbm", 1.0, src0=t, src1=t, dst=torch.empty_like(t), n=t.numel(),
                         passes=1)
    assert ei.value.status == 1
    assert ctx.serve(_trace()[:2], policy="naive", hbm_budget=1 << 30, slots=2)[1]["status"] == 0

@pytest.mark.parametrize("policy", ["usher", "sensitivity"])
def test_serve_admits_a_lone_request_the_rule_would_refuse_beside_others(ctx, policy):
    """A request that fills every wave slot (occupancy 1) and predicts 5x
    beside itself: on an idle device it is admitted (the loop would otherwise
    wait for ever), beside another it waits."""
    greedy = {"sens": {"hbm": [5.0] * 5}, "press": {"hbm": 1.0}, "occ": 1.0}
    profiles = {"triad": greedy, "gemv": greedy, "gemm": greedy}
    reqs = [dict(r, arrival_s=0.0) for r in _trace()[:4]]
    out = ctx.serve(reqs, policy=policy, bound=1.01, hbm_budget=1 << 30, slots=4, profiles=profiles)
    assert all(o["status"] == 0 for o in out)
    spans = sorted((o["admit_s"], o["end_s"]) for o in out)
    assert all(spans[i + 1][0] >= spans[i][1] - 1e-6 for i in range(len(spans) - 1))


def test_serve_rejects_bad_traces(ctx):
    from paper_2501_16909_amd import coloc
    with pytest.raises(coloc.CiError):
        ctx.serve([{"arrival_s": 1.0, "kind": "triad", "n": 10, "seed": 1},
                   {"arrival_s": 0.5, "kind": "triad", "n": 10, "seed": 2}])
    with pytest.raises(coloc.CiError):
        ctx.serve([{"arrival_s": 0.0, "kind": "gemm", "m": 8, "n": 8, "k": 12, "dtype": "bf16", "seed": 1}])
    with pytest.raises(coloc.CiError) as ei:
        ctx.serve([{"arrival_s": 0.0, "kind": "triad", "n": 1 << 26, "seed": 1}], hbm_budget=1 << 20)
    assert ei.value.status == 3
    assert ctx.serve([], policy="naive") == []
