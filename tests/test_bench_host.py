"""Host logic of the benchmark driver (no device): suite bookkeeping, the
profile combination and the pairwise slowdown model used by the estimator
and serving configurations, and the one-GPU guard."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_suite_entries_map_to_resources():
    assert bench.suite_resource("hbm") == "hbm"
    assert [bench.suite_resource(n) for n in ("hbm_read", "hbm_copy", "hbm_write")] == ["hbm"] * 3
    assert bench.suite_resource("l2_32w") == "l2" and bench.suite_resource("lds_32w") == "lds"
    assert bench.suite_resource("mfma_bf16") == "mfma_bf16"
    assert bench.suite_resource("lds_load") == "lds" and bench.suite_resource("mall_32w") == "mall"
    assert len({n for n, _ in bench.SUITE_LABELS}) == len(bench.SUITE_LABELS)


def _prof(hbm, press, wf=0.0):
    return {"sens": {"hbm": list(hbm)}, "press": {"hbm": press}, "occ": 1.0, "hbm_write_frac": wf}


def test_median_profiles_is_pointwise():
    runs = [{"k": _prof([1, 1.2, 1.5, 1.6, 2.0], 0.9)}, {"k": _prof([1, 1.4, 1.7, 1.9, 2.4], 0.7)},
            {"k": _prof([1, 1.3, 2.0, 1.7, 2.2], 0.8)}]
    m = bench.median_profiles(runs)["k"]
    assert m["sens"]["hbm"] == [1.0, 1.3, 1.7, 1.7, 2.2] and m["press"]["hbm"] == 0.8
    assert m["hbm_write_frac"] == 0.0 and m["occ"] == 1.0


def test_pair_model_product_and_pricing_switches():
    x = bench.INTENSITIES                   # 0, .25, .5, .75, 1
    base = {"v": _prof([1, 1.5, 2, 2.5, 3], 0.0, 1 / 3),
            "reader": _prof([1, 1, 1, 1, 1], 0.5, 0.0),
            "writer": _prof([1, 1, 1, 1, 1], 1.0, 1 / 3)}
    # interpolated on the victim's curve at the co-runner's pressure
    assert bench.predicted_pair_slowdown(base, "v", "reader") == 2.0
    assert bench.predicted_pair_slowdown(base, "v", "writer") == 3.0
    # read-mostly co-runners switch to the read-only curve and pressure
    read = {"v": _prof([1, 1.1, 1.2, 1.3, 1.4], 0.0), "reader": _prof([1] * 5, 0.25), "writer": _prof([1] * 5, 0.9)}
    assert np.isclose(bench.predicted_pair_slowdown(base, "v", "reader", read), 1.1)
    assert bench.predicted_pair_slowdown(base, "v", "writer", read) == 3.0
    # a co-runner that fits the Infinity Cache is priced on that curve
    mall = {k: {"sens": {"mall": [1, 1.05, 1.1, 1.15, 1.2]}, "press": {"mall": 0.5}} for k in base}
    fits = dict(bench.KIND_FOOTPRINT)
    try:
        bench.KIND_FOOTPRINT.update({"v": 1, "reader": 1, "writer": 1})
        assert np.isclose(bench.predicted_pair_slowdown(base, "v", "writer", read, mall), 1.1)
        bench.KIND_FOOTPRINT.update({"writer": 10 ** 12})
        assert bench.predicted_pair_slowdown(base, "v", "writer", read, mall) == 3.0
    finally:
        bench.KIND_FOOTPRINT.clear()
        bench.KIND_FOOTPRINT.update(fits)
    # never below 1 on any resource
    low = {"v": _prof([0.9] * 5, 0.0), "w": _prof([1] * 5, 1.0, 0.5)}
    assert bench.predicted_pair_slowdown(low, "v", "w") == 1.0
    assert len(x) == 5


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_cpu_sensitivity_leg_flags_outputs_outside_the_bound():
    """The host leg checks the sensitivity block's victims against the FP64
    oracle: the exact products pass, an entry moved by ten times its bound
    fails."""
    import oracle
    rng = np.random.default_rng(5)
    k, n = 64, 32
    a = oracle.f32_to_bf16(rng.standard_normal((16, k)).astype(np.float32)).view(np.int16)
    b = oracle.f32_to_bf16(rng.standard_normal((16, k)).astype(np.float32)).view(np.int16)
    fa, fb = oracle.bf16_to_f64(a.view(np.uint16)), oracle.bf16_to_f64(b.view(np.uint16))
    exact = np.einsum("ik,ik->i", fa, fb)
    w = oracle.f32_to_bf16(rng.standard_normal((n, k)).astype(np.float32)).view(np.int16)
    x = oracle.f32_to_bf16(rng.standard_normal(k).astype(np.float32)).view(np.int16)
    y = oracle.bf16_to_f64(w.view(np.uint16)) @ oracle.bf16_to_f64(x.view(np.uint16))
    sens = {"gemm": {"k": k, "a_rows": a, "b_cols": b, "got": exact.copy()},
            "gemv": {"w": w, "x": x, "got": y.copy()}}
    leg = bench._cpu_sensitivity_leg(sens)
    assert leg["gemm_within_bound"] and leg["gemv_within_bound"]
    bound = oracle.accumulation_bound(k + 1, np.abs(fa * fb).sum(axis=1), 2.0 ** -23)
    sens["gemm"]["got"][3] += 10 * bound[3]
    leg = bench._cpu_sensitivity_leg(sens)
    assert not leg["gemm_within_bound"] and leg["gemv_within_bound"]


def test_gemm_counter_summary_derives_rates(tmp_path):
    """The counter summariser's arithmetic on a hand-made database with the
    columns of rocprofv3's counters_collection view."""
    import sqlite3
    db = tmp_path / "g.db"
    con = sqlite3.connect(db)
    con.execute("create table counters_collection (dispatch_id int, kernel_name text, grid_size int, "
                "workgroup_size int, counter_name text, value real, start int, end int)")
    active = 240_000.0                       # cycles per XCD: 100 us at 2.4 GHz
    ctr = {"GRBM_GUI_ACTIVE": active * 8, "SQ_VALU_MFMA_BUSY_CYCLES": 0.5 * active * 1024,
           "SQ_INSTS_LDS": 48.0 * active * 256 / 1024, "SQ_WAVE_CYCLES": 1000.0, "SQ_WAIT_ANY": 250.0,
           "SQ_WAIT_INST_LDS": 20.0, "SQ_LDS_BANK_CONFLICT": 0.0, "SQ_WAVES": 2048.0, "SQ_BUSY_CYCLES": 1.0}
    for name, v in ctr.items():               # each counter split over two rows, as per-instance values are
        for half in (0.5, 0.5):
            con.execute("insert into counters_collection values (7, ?, ?, ?, ?, ?, ?, ?)",
                        ("void ci::(anonymous namespace)::gemm256d_kernel<1, 8u>(unsigned char const*)",
                         256 * 512, 512, name, v * half, 1_000, 121_000))
    con.commit()
    con.close()
    md = tmp_path / "out.md"
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--config", "gemm-counter-summary",
                        "--dbs", str(db), "--md", str(md), "--cmd", "rocprofv3 --pmc X -- python3 bench.py"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr
    row = [l for l in md.read_text().splitlines() if l.startswith("| 1 |")][0].split("|")[1:-1]
    cells = [c.strip() for c in row]
    assert cells[:6] == ["1", "120.0", "100.0", "0.500", "48.0", "0.250"]
    assert cells[6:] == ["0.020", "0", "2880000", "2048"]
    assert "`gemm256d_kernel<1, 8u>`, 256 work-groups of 512 threads" in md.read_text()


def test_reference_summary_rates(tmp_path):
    """The HBM reference summariser on a hand-made kernel table with the
    columns of rocprofv3's kernels view: unknown kernels are left out;
    rates are algorithmic bytes over the median duration, the framework's
    launches covering half the elements."""
    import sqlite3
    db = tmp_path / "t.db"
    con = sqlite3.connect(db)
    con.execute("create table kernels (name text, grid_x int, workgroup_x int, duration int, start int)")
    n = 1 << 30
    rows = [("void ci::(anonymous namespace)::stream_stressor<1u, true, 4, true>(ci::KCtrl, float const*)",
             256 * 512, 512, d) for d in (2_000_000, 2_100_000, 1_900_000)]
    rows += [("void at::native::vectorized_elementwise_kernel<4, at::native::CUDAFunctor_add<float> >(int)",
              1 << 20, 256, d) for d in (2_400_000, 2_400_000)]
    rows += [("void at::native::vectorized_elementwise_kernel<4, at::native::FillFunctor<float> >(int)",
              1 << 20, 256, 700_000)]
    rows += [("stamp_kernel(unsigned long*)", 64, 64, 900_000),            # not a reference kernel
             ("void ci::(anonymous namespace)::fill_uniform_f32(float*)", 65536 * 256, 256, 900_000),
             ("__amd_rocclr_copyBuffer", 2 * 512, 512, 3_000)]                # a small runtime copy
    for i, r in enumerate(rows):
        con.execute("insert into kernels values (?, ?, ?, ?, ?)", (*r, i))
    con.commit()
    con.close()
    md = tmp_path / "ref.md"
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--config", "reference-summary",
                        "--dbs", str(db), "--md", str(md)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr
    lines = [l for l in md.read_text().splitlines() if l.startswith("| `")]
    assert len(lines) == 3
    cells = {l.split("|")[1].strip(): [c.strip() for c in l.split("|")[2:-1]] for l in lines}
    tri = cells["`stream_stressor<1u, true, 4, true>`"]
    assert tri[1:] == ["256 x 512", "2^30", "3", "2000.0", f"{12 * n / 2_000_000:.0f}",
                       f"{12 * n / 2_000_000 / 80:.1f}"]
    add = [v for k, v in cells.items() if "add" in k][0]
    assert add[0].startswith("framework elementwise triad") and add[2:5] == ["2^29", "2", "2400.0"]
    assert add[5] == f"{12 * n / 2 / 2_400_000:.0f}"
    fill = [v for k, v in cells.items() if "Fill" in k][0]
    assert fill[5] == f"{4 * n / 2 / 700_000:.0f}"


def test_cpu_serving_leg_replays_with_a_background_load():
    """The CPU leg's discrete-event replay: two requests predicted 1x beside
    each other overlap; a background load that alone predicts 2x for each
    (above the 1.5 bound) serialises them and stretches each by 2x."""
    import bench
    prof = {"triad": {"sens": {"hbm": [1.0, 1.5, 2.0, 2.5, 3.0]}, "press": {"hbm": 0.0}, "occ": 0.25,
                      "hbm_write_frac": 1 / 3}}
    base = {"rate": 1.0, "policy": "sensitivity", "iso_s": [2.0, 2.0], "footprints": [1, 1], "budget": 1024,
            "bound": 1.5, "slots": 4, "latency_ms_p50": 0.0, "latency_ms_p99": 0.0,
            "reqs": [{"arrival_s": 0.0, "kind": "triad"}, {"arrival_s": 0.5, "kind": "triad"}]}
    loaded = dict(base, background={"press": {"hbm": 0.5}, "occ": 0.25, "hbm_write_frac": 1 / 3})
    plain, bg = bench._cpu_serving_leg({"profiles": prof, "runs": [base, loaded]})
    assert not plain["background"] and bg["background"]
    assert plain["model_colocated_fraction"] == 0.5 and bg["model_colocated_fraction"] == 0.0
    assert plain["model_latency_ms_p50"] == 2000.0          # both take 2 s, side by side
    assert bg["model_latency_ms_p50"] == 5750.0             # 4 s, then 3.5 s waiting + 4 s


def test_cpu_serving_leg_models_whole_stays_and_kernels():
    """With each request's whole stay when served alone (iso_span_s), the
    model's latencies use it; the kernel-only model uses iso_s."""
    import bench
    prof = {"triad": {"sens": {"hbm": [1.0] * 5}, "press": {"hbm": 0.0}, "occ": 0.25}}
    run = {"rate": 1.0, "policy": "naive", "iso_s": [2.0, 2.0], "iso_span_s": [3.0, 3.0], "footprints": [1, 1],
           "budget": 1024, "bound": 1.5, "slots": 1, "latency_ms_p50": 0.0, "latency_ms_p99": 0.0,
           "reqs": [{"arrival_s": 0.0, "kind": "triad"}, {"arrival_s": 0.0, "kind": "triad"}]}
    (r,) = bench._cpu_serving_leg({"profiles": prof, "runs": [run]})
    assert (r["model_kernel_latency_ms_p50"], r["model_kernel_latency_ms_p99"]) == (3000.0, 3980.0)
    assert (r["model_latency_ms_p50"], r["model_latency_ms_p99"]) == (4500.0, 5970.0)


def test_equivalent_duty():
    """A co-runner's pressure on the duty axis: the stressor duty whose
    standalone rate matches its use, linear between measured duty levels."""
    import bench
    table = {10: 0.2, 25: 0.5, 50: 0.8, 75: 0.9, 100: 1.0}
    f = lambda x: bench.equivalent_duty(x, table, 1.0)
    assert f(0.0) == 0.0 and f(0.2) == pytest.approx(0.1) and f(0.8) == pytest.approx(0.5)
    assert f(0.35) == pytest.approx(0.175)          # halfway between duty 10 and 25
    assert f(0.95) == pytest.approx(0.875)
    assert f(1.0) == 1.0 and f(1.5) == 1.0           # at or beyond the full rate
    assert bench.equivalent_duty(0.4, {50: 8.0, 100: 10.0}, 10.0) == pytest.approx(0.25)   # rates in any unit
    # a non-increasing measurement does not fold the table back
    g = bench.equivalent_duty(0.47, {25: 0.5, 50: 0.45, 100: 1.0}, 1.0)
    assert 0.0 < g <= 0.25


def test_trace_summary_lists_kernels_inside_a_long_launch(tmp_path):
    """trace-summary --window-ms: a launch longer than the threshold is
    listed with the kernels that ran entirely inside its window."""
    import sqlite3
    db = tmp_path / "t.db"
    con = sqlite3.connect(db)
    con.execute("create table kernels (name text, grid_x int, workgroup_x int, duration int, start int, end int)")
    rows = [("held_stressor", 256 * 512, 512, 0, 3_000_000_000),     # 3 s
            ("request", 1024, 256, 1_000_000, 1_000_100), ("request", 1024, 256, 2_000_000, 2_000_100),
            ("after", 64, 64, 3_100_000_000, 3_100_000_100)]
    con.executemany("insert into kernels values (?, ?, ?, ?, ?, ?)",
                    [(n, g, w, e - s, s, e) for n, g, w, s, e in rows])
    con.commit()
    con.close()
    md = tmp_path / "s.md"
    subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--config", "trace-summary", "--dbs", str(db),
                    "--window-ms", "1000", "--top", "2", "--md", str(md), "--cmd", "x"], check=True,
                   capture_output=True)
    text = md.read_text()
    assert "lasting 3000.0 ms; kernels that started and ended inside its window: 2" in text
    assert "- `request`: 2" in text and "`after`" not in text.split("lasting")[1]
    assert "(2 of 3 kernel and launch-shape rows, by total time.)" in text
