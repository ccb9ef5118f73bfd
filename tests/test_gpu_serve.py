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


def _oracle_check(q, served):
    s = q["seed"]
    if q["kind"] == "triad":
        b = synth.uniform_f32(s, q["n"])
        c = synth.uniform_f32(s + 1, q["n"])
        want = oracle.triad_f32(b, c)
        assert served["checksum_bits"] == oracle.bitsum_u32(want)
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


def test_serve_naive_overlaps_and_matches_isolated(ctx):
    reqs = _trace()
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
    # same result alone and in the mix (bit for bit), and against the oracle
    for q, o in zip(reqs, out):
        alone = ctx.serve([dict(q, arrival_s=0.0)], policy="naive", hbm_budget=1 << 30, slots=1)[0]
        assert alone["checksum_bits"] == o["checksum_bits"], q
        _oracle_check(q, o)


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
