#!/usr/bin/env python3
"""Benchmark of the stressor suite and colocation harness on one MI355X.

Default (one JSON line on stdout): a step is one pass of the standalone
stressor suite -- HBM triad over FP32 N = 2^30, L2 over 2 MiB, Infinity Cache
over 128 MiB, vL1D over 16 KiB, LDS over 64 KiB per work-group, FP32 FMA
chains of 4096 steps, FP32/BF16/FP8 matrix-core loops, a pointer chase over a
random 2^24 cycle, 10^6 empty 64-thread work-groups -- plus one colocated
triad pair (victim and stressor both a = b + 3c over N = 2^22).  `value` is
the HBM stressor's bandwidth; every stressor's rate and fraction of peak and
the pair's slowdown ride along in the same line.

Other workloads, each its own JSON line(s), with --config: sweep,
precision, serve, pollution, bandwidth, ilp, pairs, ldsstride, estimator,
decode, queues, hbm_mix, chase-latency; counters, suite-counters, lds-counters,
gemm-counters and hbm-references are short runs for hardware-counter
passes or a kernel trace, and the
*-summary configurations turn their rocprofv3 databases into the files
under profiles/ (no GPU).  One GPU only: --gpus N with N > 1 exits with a
message.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("victim slowdown per resource vs intensity; stressor % of peak (HBM GB/s, TFLOPS)")
# stressor workspace: control words and records for up to 16 work-groups per CU on 256 CUs
WS_BYTES = 4096 + 256 * 16 * 48


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sha_of(*paths):
    h = hashlib.sha256()
    for path in paths:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


# sources the HBM stressor's machine code is built from
HBM_KERNEL_SOURCES = [os.path.join("paper_2501_16909_amd", "csrc", f) for f in ("k_memory.hip", "stressor_dev.h")]


# --------------------------------------------------------------------------
def suite_resource(name: str) -> str:
    """Resource of a suite entry: the HBM mixes (hbm_read, ...) are the HBM
    stressor with another knob; *_32w entries are a stressor in its
    32-waves-per-CU shape instead of its colocation default."""
    if name.startswith("hbm_"):
        return "hbm"
    if name.startswith("mall_"):
        return "mall"
    if name.startswith("lds_"):
        return "lds"
    return name[:-4] if name.endswith("_32w") else name


# The suite's entries in launch order, with the label the counter summary uses.
SUITE_LABELS = [
    ("hbm", "HBM triad N=2^30"), ("hbm_read", "HBM read-only N=2^30"), ("hbm_copy", "HBM copy N=2^30"),
    ("hbm_write", "HBM write-only N=2^30"), ("l2", "L2 2 MiB (3 x 512 per CU)"),
    ("l2_32w", "L2 2 MiB (2 x 1024 per CU)"), ("mall", "Infinity Cache 128 MiB read"),
    ("mall_write", "Infinity Cache 128 MiB write-only"), ("mall_32w", "Infinity Cache 128 MiB read, 2 x 1024 per CU"),
    ("vl1d", "vL1D 16 KiB"),
    ("lds", "LDS copy vec4 stride 1 (1 WG of 16 waves per CU)"), ("lds_32w", "LDS copy, 2 WGs per CU"),
    ("lds_load", "LDS load-only vec4 stride 1"), ("lds_load_32w", "LDS load-only, 2 WGs per CU"),
    ("valu_f32", "VALU FMA ILP 8"),
    ("valu_f64", "VALU FP64 multiply ILP 4"), ("mfma_f32", "MFMA FP32"), ("mfma_bf16", "MFMA BF16"),
    ("mfma_fp8", "MFMA FP8"), ("ptrchase", "pointer chase 2^24"), ("dispatch", "dispatch 10^6 WGs")]


class Suite:
    """Device buffers and the fixed-work form of every stressor."""

    def __init__(self, ctx, dev):
        import torch
        import synth
        self.ctx, self.dev = ctx, dev
        T = lambda x: torch.from_numpy(np.require(x, requirements=["C", "W"])).to(dev)
        n = 1 << 30
        self.n_hbm = n
        self.hb = torch.empty(n, dtype=torch.float32, device=dev)
        self.hc = torch.empty_like(self.hb)
        self.ha = torch.empty_like(self.hb)
        synth.device_fill_uniform_f32(self.hb.data_ptr(), n, synth.seed_for(1, synth.BUF_B))
        synth.device_fill_uniform_f32(self.hc.data_ptr(), n, synth.seed_for(1, synth.BUF_C))
        self.l2 = torch.empty(1 << 19, dtype=torch.int32, device=dev)
        self.l1 = torch.empty(1 << 12, dtype=torch.int32, device=dev)
        synth.device_fill_u32(self.l2.data_ptr(), 1 << 19, synth.seed_for(1, synth.BUF_CACHE))
        synth.device_fill_u32(self.l1.data_ptr(), 1 << 12, synth.seed_for(1, synth.BUF_CACHE) + 2)
        # Infinity Cache: two 64 MiB arrays (128 MiB, 16 MiB per XCD slot) and an output
        self.n_mall = 1 << 24
        self.mb = torch.empty(self.n_mall, dtype=torch.float32, device=dev)
        self.mc, self.ma = torch.empty_like(self.mb), torch.empty_like(self.mb)
        synth.device_fill_uniform_f32(self.mb.data_ptr(), self.n_mall, synth.seed_for(1, synth.BUF_CACHE) + 1)
        synth.device_fill_uniform_f32(self.mc.data_ptr(), self.n_mall, synth.seed_for(1, synth.BUF_CACHE) + 3)
        self.win = T(synth.u32(synth.seed_for(1, synth.BUF_LDS), 8192).view(np.int32))
        self.valu_out = torch.empty(256 * 4 * 256 * 8, dtype=torch.float32, device=dev)
        ones = {"f32": (np.ones((32, 2), np.float32), np.ones((2, 32), np.float32)),
                "bf16": (np.full((32, 16), 0x3F80, np.int16), np.full((16, 32), 0x3F80, np.int16)),
                "fp8": (np.full((32, 64), 0x38, np.uint8), np.full((64, 32), 0x38, np.uint8))}
        self.mf = {k: (T(a), T(b)) for k, (a, b) in ones.items()}
        self.mf_out = torch.empty(256 * 2 * 4 * 4 * 1024, dtype=torch.float32, device=dev)
        self.chase = T(synth.random_cycle_u32(synth.seed_for(1, synth.BUF_CHASE), 1 << 24).view(np.int32))
        self.chase_end = torch.empty(256 * 256 * 4, dtype=torch.int32, device=dev)
        self.count = torch.zeros(1, dtype=torch.int64, device=dev)
        # colocated triad pair (N = 2^22): victim and an identical stressor
        m = 1 << 22
        self.vb = torch.empty(m, dtype=torch.float32, device=dev)
        self.vc, self.va = torch.empty_like(self.vb), torch.empty_like(self.vb)
        self.sb, self.sc, self.sa = (torch.empty_like(self.vb) for _ in range(3))
        for t, s in ((self.vb, synth.BUF_B), (self.vc, synth.BUF_C), (self.sb, synth.BUF_B2),
                     (self.sc, synth.BUF_C2)):
            synth.device_fill_uniform_f32(t.data_ptr(), m, synth.seed_for(0, s))
        torch.cuda.synchronize()
        self.ws = torch.empty(WS_BYTES, dtype=torch.uint8, device=dev)
        from paper_2501_16909_amd.coloc import HBM_MIX as mix
        self.items = [
            ("hbm", dict(src0=self.hb, src1=self.hc, dst=self.ha, n=n, passes=1), "GB/s", 1e9),
            ("hbm_read", dict(src0=self.hb, src1=self.hc, n=n, passes=1, knob=mix["read"]), "GB/s", 1e9),
            ("hbm_copy", dict(src0=self.hb, dst=self.ha, n=n, passes=1, knob=mix["copy"]), "GB/s", 1e9),
            ("hbm_write", dict(dst=self.ha, n=n, passes=1, knob=mix["write"]), "GB/s", 1e9),
            ("l2", dict(src0=self.l2, n=1 << 19, passes=32), "TB/s", 1e12),
            ("l2_32w", dict(src0=self.l2, n=1 << 19, passes=32, wg_per_cu=2, threads=1024), "TB/s", 1e12),
            ("mall", dict(src0=self.mb, src1=self.mc, n=self.n_mall, passes=60), "TB/s", 1e12),
            ("mall_write", dict(dst=self.ma, n=self.n_mall, passes=240, knob=mix["write"]), "TB/s", 1e12),
            ("mall_32w", dict(src0=self.mb, src1=self.mc, n=self.n_mall, passes=60, wg_per_cu=2, threads=1024),
             "TB/s", 1e12),
            ("vl1d", dict(src0=self.l1, n=1 << 12, passes=4000), "TB/s", 1e12),
            ("lds", dict(src0=self.win, passes=10), "TB/s", 1e12),
            ("lds_32w", dict(src0=self.win, passes=10, wg_per_cu=2), "TB/s", 1e12),
            ("lds_load", dict(src0=self.win, passes=20, access=1), "TB/s", 1e12),
            ("lds_load_32w", dict(src0=self.win, passes=20, access=1, wg_per_cu=2), "TB/s", 1e12),
            ("valu_f32", dict(dst=self.valu_out, iters=4096, passes=4, fa=1 - 2 ** -12, fb=2 ** -12), "TFLOP/s", 1e12),
            ("valu_f64", dict(dst=self.valu_out, iters=4096, passes=4, fa=1 - 2 ** -12), "TFLOP/s", 1e12),
            ("mfma_f32", dict(src0=self.mf["f32"][0], src1=self.mf["f32"][1], dst=self.mf_out, iters=2048, passes=2), "TFLOP/s", 1e12),
            ("mfma_bf16", dict(src0=self.mf["bf16"][0], src1=self.mf["bf16"][1], dst=self.mf_out, iters=2048, passes=2), "TFLOP/s", 1e12),
            ("mfma_fp8", dict(src0=self.mf["fp8"][0], src1=self.mf["fp8"][1], dst=self.mf_out, iters=2048, passes=2), "TFLOP/s", 1e12),
            ("ptrchase", dict(src0=self.chase, n=1 << 24, dst=self.chase_end, iters=512, passes=1), "Ghop/s", 1e9),
            ("dispatch", dict(iters=1000000, passes=1), "MWG/s", 1e6),
        ]
        assert [it[0] for it in self.items] == [n for n, _ in SUITE_LABELS]

    def step(self, acc, warm: int = 0):
        for name, opts, unit, scale in self.items:
            res = suite_resource(name)
            for _ in range(warm):   # untimed launches of the same stressor first
                self.ctx.stressor(res, 1.0, ws=self.ws, **opts).stop()
            st = self.ctx.stressor(res, 1.0, ws=self.ws, **opts)
            rep = st.stop()
            rate = rep.units / (rep.kernel_ns * 1e-9)
            a = acc.setdefault(name, {"unit": unit, "scale": scale, "rates": [], "kernel_ns": [],
                                      "pct": [], "units": rep.units})
            a["rates"].append(rate)
            a["kernel_ns"].append(rep.kernel_ns)
            a["pct"].append(100.0 * rate / self.ctx.peak(res) if self.ctx.peak(res) > 0 else None)
        # colocated triad pair (shared CUs and disjoint halves)
        d = self.ctx.triad_desc(self.vb, self.vc, self.va, passes=10)
        so = [dict(src0=self.sb, src1=self.sc, dst=self.sa, n=1 << 22)]
        for placement, x in (("shared", 1.0), ("disjoint", 0.5)):
            cell = self.ctx.measure_sensitivity(d, ["hbm"], so, [x], reps=3, warmups=1,
                                                placement=placement, ws=self.ws)[0]
            acc.setdefault("pair_" + placement, []).append(cell)


def hbm_traffic():
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "hbm_triad_n2e30_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        c = json.load(f)
    if c.get("kernel_source_sha") != sha_of(*[os.path.join(ROOT, p) for p in HBM_KERNEL_SOURCES]):
        return None
    return c.get("traffic_bytes_per_launch")


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _host_threads() -> int:
    """Threads the CPU baseline may use: the cores this process may run on,
    capped by OMP_NUM_THREADS when the environment sets a share."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    cap = os.environ.get("OMP_NUM_THREADS")
    if cap and cap.isdigit() and int(cap) > 0:
        n = min(n, int(cap))
    return max(1, n)


def cpu_baseline(host=None, prec=None, serve=None, sens=None):
    """The oracle on the host CPU, beside the GPU legs of the same run.

    triad: the oracle's two-rounding triad over the headline's N = 2^30
      arrays (copied from the device, the same bits), once on one thread and
      repeatedly on every host thread the process may use;
    precision: the FP64 oracle on the precision legs' 4096 sampled entries,
      timed, and the GPU outputs' errors against it (per dtype: kernel error
      against the quantised inputs, total error against the FP32 inputs, and
      the largest error over its bound);
    serving: the admission rule replayed in the oracle's discrete-event
      model on each served trace with the requests' isolated service times:
      the latency it predicts next to the one the GPU loop measured;
    sensitivity: the sensitivity block's GEMV (whole) and GEMM (sampled)
      outputs against the FP64 oracle, timed."""
    import oracle
    import synth
    out = {"kind": "oracle", "unit": "GB/s"}
    threads = _host_threads()
    if host is not None:
        b, c = host
        n = b.size
    else:          # no device arrays (a bounded host-only sample)
        n = 1 << 26
        b = synth.uniform_f32(synth.seed_for(1, synth.BUF_B), n)
        c = synth.uniform_f32(synth.seed_for(1, synth.BUF_C), n)
    a = np.empty_like(b)
    oracle.triad_f32(b[:1024], c[:1024])
    t0 = time.perf_counter()
    oracle.triad_f32_threads(b, c, 1, out=a)
    t1 = time.perf_counter() - t0
    reps, used = 0, threads
    t0 = time.perf_counter()
    while True:
        _, used = oracle.triad_f32_threads(b, c, threads, out=a)
        reps += 1
        if time.perf_counter() - t0 > 5.0 and reps >= 2:
            break
    tall = (time.perf_counter() - t0) / reps
    out.update({"value": round(12.0 * n / tall / 1e9, 3), "cores": used,
                "value_1t": round(12.0 * n / t1 / 1e9, 3), "nproc": os.cpu_count(),
                "cpu_model": _cpu_model(), "n": int(n),
                "sample": f"C oracle triad a = b + 3c (two FP32 roundings) over N = {n} FP32 elements: "
                          f"one pass on 1 thread ({t1:.2f} s), {reps} passes on {used} threads "
                          f"({tall:.2f} s each)"})
    del a
    legs = {}
    if sens is not None:
        legs["sensitivity"] = _cpu_sensitivity_leg(sens)
    if prec is not None:
        legs["precision"] = _cpu_precision_leg(prec)
    if serve is not None:
        legs["serving"] = _cpu_serving_leg(serve)
    if legs:
        out["legs"] = legs
    return out


def _cpu_sensitivity_leg(sens):
    """The sensitivity block's victims against the FP64 oracle: the GEMV's
    whole output and the GEMM's sampled entries, each within its FP32
    accumulation bound, with the oracle's time."""
    import oracle
    g, v = sens["gemm"], sens["gemv"]
    t0 = time.perf_counter()
    fa, fb = oracle.bf16_to_f64(g["a_rows"].view(np.uint16)), oracle.bf16_to_f64(g["b_cols"].view(np.uint16))
    pair = np.arange(len(fa))
    want = oracle.gemm_entries_f64(fa, fb, pair, pair)
    t_gemm = time.perf_counter() - t0
    absg = oracle.gemm_entries_f64(np.abs(fa), np.abs(fb), pair, pair)
    bound_g = oracle.accumulation_bound(g["k"] + 1, absg, 2.0 ** -23)
    t0 = time.perf_counter()
    fw, fx = oracle.bf16_to_f64(v["w"].view(np.uint16)), oracle.bf16_to_f64(v["x"].view(np.uint16))
    want_v = oracle.gemv_f64(fw, fx)
    t_gemv = time.perf_counter() - t0
    bound_v = oracle.accumulation_bound(fw.shape[1] + 1, np.abs(fw) @ np.abs(fx), 2.0 ** -24)
    err_g, err_v = np.abs(g["got"] - want), np.abs(v["got"] - want_v)
    return {"sample": f"GEMM BF16 {g['k']}^3 on {len(fa)} fixed-seed entries; GEMV BF16 "
                      f"{fw.shape[0]} x {fw.shape[1]} whole",
            "gemm_within_bound": bool(np.all(err_g <= bound_g)),
            "gemm_err_max_over_bound": float((err_g / bound_g).max()),
            "gemv_within_bound": bool(np.all(err_v <= bound_v)),
            "gemv_err_max_over_bound": float((err_v / bound_v).max()),
            "oracle_seconds": {"gemm_sampled": round(t_gemm, 3), "gemv_full": round(t_gemv, 3)},
            "oracle_gemm_entries_per_s": round(len(fa) / t_gemm, 1)}


def _cpu_precision_leg(prec):
    """Errors of the sampled GPU GEMM outputs against the FP64 oracle."""
    import oracle
    res = {"sample": f"{len(prec['rows'])} fixed-seed entries of C = A B^T, M = N = K = {prec['k']}",
           "dtypes": {}}
    t0 = time.perf_counter()
    exact = oracle.gemm_entries_f64(prec["a_rows"], prec["b_cols"], prec["pair"], prec["pair"])
    absx = oracle.gemm_entries_f64(np.abs(prec["a_rows"]), np.abs(prec["b_cols"]), prec["pair"], prec["pair"])
    t_exact = time.perf_counter() - t0
    for dt, d in prec["dtypes"].items():
        if dt == "f32":
            fa, fb = d["qa"].astype(np.float64), d["qb"].astype(np.float64)
        elif dt == "bf16":
            fa, fb = oracle.bf16_to_f64(d["qa"].view(np.uint16)), oracle.bf16_to_f64(d["qb"].view(np.uint16))
        else:
            fa, fb = oracle.e4m3_to_f64(d["qa"]), oracle.e4m3_to_f64(d["qb"])
        s = d["sa"] * d["sb"]
        kern = s * oracle.gemm_entries_f64(fa, fb, prec["pair"], prec["pair"])
        kabs = s * oracle.gemm_entries_f64(np.abs(fa), np.abs(fb), prec["pair"], prec["pair"])
        if dt == "fp8":
            bound = oracle.mfma_fp8_error_bound(d["qa"], d["qb"], s)
        else:
            bound = s * oracle.accumulation_bound(prec["k"] + 1, kabs / s, 2.0 ** -23)
        got = d["got"]
        res["dtypes"][dt] = {
            "kernel_err_max_rel_absprod": float(np.max(np.abs(got - kern) / kabs)),
            "kernel_err_normwise": float(np.linalg.norm(got - kern) / np.linalg.norm(kern)),
            "kernel_err_max_over_bound": float(np.max(np.abs(got - kern) / bound)),
            "total_err_max_rel_absprod": float(np.max(np.abs(got - exact) / absx)),
            "total_err_normwise": float(np.linalg.norm(got - exact) / np.linalg.norm(exact))}
    res["oracle_entries_per_s"] = round(len(prec["rows"]) / t_exact, 1)
    res["oracle_full_gemm_s_extrapolated"] = round(prec["k"] ** 2 / (len(prec["rows"]) / t_exact), 1)
    return res


def _cpu_serving_leg(serve):
    """The admission rule in the oracle's discrete-event model, fed the
    isolated service times the GPU measured, next to the GPU's latencies.
    Two service times per request: its kernel alone (model_kernel_*), and
    its whole stay in the loop when served alone (model_*: input
    generation, kernel, checksum and retirement), which is what the GPU's
    latencies include."""
    import oracle
    out = []
    for run in serve["runs"]:
        prof, reqs = serve["profiles"], run["reqs"]
        f32 = lambda v: float(np.float32(v))
        names = ["hbm", "l2", "mall", "vl1d", "lds", "valu_f32", "mfma_f32", "mfma_bf16", "mfma_fp8", "ptrchase",
                 "dispatch", "occupancy", "valu_f64"]
        jobs = []
        for q in reqs:
            p = prof[q["kind"]]
            job = {"sens": [[f32(v) for v in p["sens"].get(r, [1.0] * 5)] for r in names],
                   "press": [f32(p["press"].get(r, 0.0)) for r in names], "occ": f32(p["occ"]),
                   "bytes": run["footprints"][len(jobs)], "hbm_write_frac": f32(p.get("hbm_write_frac", 1.0)),
                   "press_hbm_read": f32(p.get("press_hbm_read", 0.0))}
            if p.get("sens_hbm_read"):
                job["sens_hbm_read"] = [f32(v) for v in p["sens_hbm_read"]]
            jobs.append(job)
        bg = None
        if run.get("background"):
            b = run["background"]
            bg = {"press": [f32(b["press"].get(r, 0.0)) for r in names], "occ": f32(b["occ"]),
                  "hbm_write_frac": f32(b.get("hbm_write_frac", 1.0)),
                  "press_hbm_read": f32(b.get("press_hbm_read", 0.0))}
        t0 = time.perf_counter()
        arrivals = [q["arrival_s"] for q in reqs]
        sim_k = oracle.simulate_admission(arrivals, jobs, run["iso_s"], run["policy"], run["budget"],
                                          run["bound"], run["slots"], slowed=True, background=bg)
        sim = oracle.simulate_admission(arrivals, jobs, run.get("iso_span_s", run["iso_s"]), run["policy"],
                                        run["budget"], run["bound"], run["slots"], slowed=True, background=bg)
        dt = time.perf_counter() - t0
        lat_k = np.array([o["end"] - a for o, a in zip(sim_k, arrivals)])
        lat = np.array([o["end"] - a for o, a in zip(sim, arrivals)])
        out.append({"rate_per_s": run["rate"], "policy": run["policy"], "background": bg is not None,
                    "requests": len(reqs),
                    "model_latency_ms_p50": round(float(np.percentile(lat, 50)) * 1e3, 3),
                    "model_latency_ms_p99": round(float(np.percentile(lat, 99)) * 1e3, 3),
                    "model_kernel_latency_ms_p50": round(float(np.percentile(lat_k, 50)) * 1e3, 3),
                    "model_kernel_latency_ms_p99": round(float(np.percentile(lat_k, 99)) * 1e3, 3),
                    "gpu_latency_ms_p50": run["latency_ms_p50"], "gpu_latency_ms_p99": run["latency_ms_p99"],
                    "model_colocated_fraction": round(float(np.mean([bool(o["corunners"]) for o in sim])), 3),
                    "oracle_seconds": round(dt, 2)})
    return out


# the compact sensitivity block of the default run: both sweep victims against
# the resources each kind of workload loads, at CU intensity 0, 50 and 100 %
SENS_RES = ["hbm", "l2", "mall", "lds", "valu_f32", "mfma_bf16", "ptrchase"]
SENS_X = [0.0, 0.5, 1.0]


def sensitivity_block(ctx, dev, reps, ws, keep_host=False):
    """Victim slowdown per resource and intensity (shared CUs) for the BF16
    GEMM 4096^3 and the BF16 GEMV 8192^2 of the sensitivity sweep, each cell
    with its bootstrap 95 % interval and the stressor's share of its peak.
    With keep_host, also returns the victims' quantised inputs and outputs
    (the GEMM on 4096 fixed-seed entries, the GEMV whole) for the CPU leg:
    every cell's colocated output equals its alone output, so these are the
    outputs of every run."""
    import torch
    import synth
    ops = stressor_operands(dev)
    victims = sweep_victims(ctx, dev)
    nan = lambda v: v != v
    out = {"intensities": SENS_X, "reps": reps, "placement": "shared", "victims": {}}
    for vname in ("gemm_bf16_4096", "gemv_bf16_8192"):
        cells = ctx.measure_sensitivity(victims[vname], SENS_RES, [ops[r] for r in SENS_RES], SENS_X, reps=reps,
                                        warmups=2, ws=ws, deadline_ms=200)
        tab = {}
        for i, r in enumerate(SENS_RES):
            row = cells[i * len(SENS_X):(i + 1) * len(SENS_X)]
            tab[r] = {"slowdown": [None if nan(c["slowdown"]) else round(c["slowdown"], 3) for c in row],
                      "ci95": [None if nan(c["slowdown_ci_lo"]) else
                               [round(c["slowdown_ci_lo"], 3), round(c["slowdown_ci_hi"], 3)] for c in row],
                      "stressor_pct_peak": [round(c["stressor_pct_peak"], 1) for c in row],
                      "starved_lower_bound": [bool(c["timed_out"]) for c in row],
                      "valid": [bool(c["window_covered"] and c["output_equal"] and not c["queue_unresolved"])
                                for c in row]}
        out["victims"][vname] = {"t_alone_us": round(float(np.median([c["t_alone_ns"] for c in cells])) / 1e3, 2),
                                 "cells": tab}
        log(f"sensitivity {vname}: " + ", ".join(f"{r}={tab[r]['slowdown']}" for r in tab))
    out["queue_pair_check"] = ctx.queue_stats()
    host = None
    if keep_host:
        qa, qb, c = victims["gemm_bf16_4096"]._keep
        m = c.shape[0]
        idx = synth.words(4243, 4096)
        rows = (idx % np.uint64(m)).astype(np.int64)
        cols = ((idx >> np.uint64(32)) % np.uint64(m)).astype(np.int64)
        rt, ct = torch.from_numpy(rows).to(dev), torch.from_numpy(cols).to(dev)
        w3, qx, y = victims["gemv_bf16_8192"]._keep
        n = y.numel()
        host = {"gemm": {"k": m, "a_rows": qa.view(m, m)[rt].cpu().numpy(), "b_cols": qb.view(m, m)[ct].cpu().numpy(),
                         "got": c[rt, ct].double().cpu().numpy()},
                "gemv": {"w": w3[:n * n].view(n, n).cpu().numpy(), "x": qx.cpu().numpy(),
                         "got": y.double().cpu().numpy()}}
    del ops, victims
    return out, host


def precision_block(ctx, dev, keep_host):
    """GEMM 8192^3 from N(0, 1) in FP32, BF16 and FP8 (per-tensor scale):
    time and rate per dtype; the sampled entries (and the operands' rows
    that produce them) go to the CPU leg for the error against FP64."""
    import torch
    import synth
    m = 8192
    ha = synth.normal_f32(synth.seed_for(3, synth.BUF_GEMM_A), m * m).reshape(m, m)
    hb = synth.normal_f32(synth.seed_for(3, synth.BUF_GEMM_B), m * m).reshape(m, m)
    a = torch.from_numpy(ha).to(dev)
    b = torch.from_numpy(hb).to(dev)
    c = torch.empty((m, m), dtype=torch.float32, device=dev)
    idx = synth.words(4242, 4096)
    rows = (idx % np.uint64(m)).astype(np.int64)
    cols = ((idx >> np.uint64(32)) % np.uint64(m)).astype(np.int64)
    host = {"k": m, "rows": rows, "cols": cols, "pair": np.arange(len(rows)),
            "a_rows": ha[rows].copy(), "b_cols": hb[cols].copy(), "dtypes": {}}
    summary = {}
    rt, ct = torch.from_numpy(rows).to(dev), torch.from_numpy(cols).to(dev)
    for dt in ("f32", "bf16", "fp8"):
        if dt == "f32":
            qa, qb, sa, sb = a, b, 1.0, 1.0
        else:
            qa, sa = ctx.quantize(a, dt)
            qb, sb = ctx.quantize(b, dt)
        d = ctx.gemm_desc(qa, qb, c, dt, m, m, m, sa, sb)
        for _ in range(5):      # untimed: the rate rises over a process's first launches
            ctx.victim_run(d)
        times = [ctx.victim_run(d).time_ns for _ in range(10)]
        t = float(np.median(times))
        summary[dt] = {"time_ms": round(t / 1e6, 3), "tflops": round(2.0 * m ** 3 / t / 1e3, 1),
                       "pct_of_peak": round(100 * 2.0 * m ** 3 / (t * 1e-9) / ctx.peak("mfma_" + dt), 1)}
        if keep_host:
            host["dtypes"][dt] = {"qa": qa.index_select(0, rt).cpu().numpy(), "qb": qb.index_select(0, ct).cpu().numpy(),
                                  "sa": sa, "sb": sb, "got": c[rt, ct].cpu().numpy().astype(np.float64)}
        log(f"precision {dt}: {summary[dt]}")
    del a, b, c
    torch.cuda.empty_cache()
    return summary, host


def background_load(ctx, dev, duty, mix="triad"):
    """An HBM stressor for serve_run_background, in the triad or the
    read-only mix: its operands (2^28-element FP32 arrays, 1 GiB each, far
    beyond the Infinity Cache), a workspace, and its load as the admission
    rules see it, in the duty-axis profiles' units: the triad at duty d is
    the triad curves' point d; the read-only mix at duty d is the read-only
    curves' point d and, for the triad curves, the triad duty whose
    standalone byte rate matches its own (equivalent_duty).  Both hold one
    512-thread work-group per CU (8 of 32 wave slots)."""
    import torch
    import synth
    from paper_2501_16909_amd.coloc import HBM_MIX
    n = 1 << 28
    hb = torch.empty(n, dtype=torch.float32, device=dev)
    hc, ha = torch.empty_like(hb), torch.empty_like(hb)
    synth.device_fill_uniform_f32(hb.data_ptr(), n, synth.seed_for(4, synth.BUF_B))
    synth.device_fill_uniform_f32(hc.data_ptr(), n, synth.seed_for(4, synth.BUF_C))
    torch.cuda.synchronize()
    triad = dict(src0=hb, src1=hc, dst=ha, n=n)
    ws = torch.empty(WS_BYTES, dtype=torch.uint8, device=dev)
    if mix == "triad":
        return triad, ws, {"press": {"hbm": duty / 100.0}, "occ": 0.25, "hbm_write_frac": HBM_WRITE_FRAC["triad"]}

    def rate(o, **kw):   # median of three launches after an untimed one
        run = lambda: ctx.stressor("hbm", 1.0, ws=ws, passes=1, **o, **kw).stop()
        run()
        return float(np.median([(lambda r: r.units / r.kernel_ns)(run()) for _ in range(3)]))
    full = rate(triad)
    table = {d: rate(triad, duty=d) for d in DUTIES}
    ops = dict(src0=hb, src1=hc, n=n, knob=HBM_MIX["read"])
    part = rate(ops, duty=duty)
    return ops, ws, {"press": {"hbm": equivalent_duty(part / full, table, full)}, "occ": 0.25,
                     "hbm_write_frac": 0.0, "press_hbm_read": duty / 100.0}


def serving_block(ctx, args, keep_host):
    """The serving loop on the serving configuration's traffic: Poisson arrivals of BF16
    GEMM / BF16 GEMV / FP32 triad requests, naive against sensitivity-aware
    admission (duty-axis profiles measured here, read/write-aware HBM
    pricing), 60 s at 200 requests/s and 10 s at 1000/s.  Every request is
    also served alone (one slot, in arrival order) for its isolated service
    time and result: slowdowns are over all requests, and every result must
    equal its isolated one bit for bit.  The 1000/s trace is also served on
    a loaded device: an HBM triad stressor on every CU at 25 % duty held for
    the whole run (serve_run_background), its load in the admission rules."""
    from paper_2501_16909_amd import coloc
    profiles = library_profiles(serve_profiles(ctx, args, axis="duty"),
                                serve_profiles(ctx, args, axis="duty", hbm_mix="read", res=("hbm",)))
    budget, slots = 32 << 30, 4
    summary = {"config": {"workload": "Poisson arrivals, 1/3 each BF16 GEMM n~logU[512,8192], BF16 GEMV "
                                      "n~logU[4096,16384], FP32 triad N~logU[2^20,2^28]",
                          "slots": slots, "hbm_budget_gib": budget >> 30, "bound": args.bound,
                          "profile_axis": "duty", "hbm_pricing": "read/write-aware"},
               "runs": []}
    host = {"profiles": profiles, "runs": []}
    for lam, seconds in ((200.0, args.serve_seconds), (1000.0, max(2.0, args.serve_seconds / 6))):
        reqs = serve_trace(lam, seconds, 31337 + int(lam))
        iso = ctx.serve([dict(r, arrival_s=0.0) for r in reqs], policy="naive", hbm_budget=budget, slots=1)
        iso_ns = np.array([o["service_ns"] for o in iso])
        iso_span = [o["end_s"] - o["admit_s"] for o in iso]   # inputs, kernel, checksum, retirement
        for policy in ("naive", "sensitivity"):
            t0 = time.perf_counter()
            res = ctx.serve(reqs, policy=policy, bound=args.bound, hbm_budget=budget, slots=slots,
                            profiles=profiles)
            wall = time.perf_counter() - t0
            lat = np.array([r["end_s"] - r["arrival_s"] for r in res])
            slow = np.array([r["service_ns"] for r in res]) / iso_ns
            equal = all(r["checksum_bits"] == i["checksum_bits"] for r, i in zip(res, iso))
            run = {"rate_per_s": lam, "seconds": seconds, "policy": policy, "requests": len(reqs),
                   "latency_ms_p50": round(float(np.percentile(lat, 50)) * 1e3, 3),
                   "latency_ms_p99": round(float(np.percentile(lat, 99)) * 1e3, 3),
                   "throughput_req_s": round(len(reqs) / max(r["end_s"] for r in res), 1),
                   "slowdown_p50": round(float(np.percentile(slow, 50)), 3),
                   "slowdown_p99": round(float(np.percentile(slow, 99)), 3),
                   "slowdown_over": "every request (service in the mix / service alone)",
                   "results_equal_isolated": bool(equal), "wall_s": round(wall, 1)}
            summary["runs"].append(run)
            log(f"serve {lam}/s {policy}: {run}")
            if keep_host:
                host["runs"].append({"rate": lam, "policy": policy, "reqs": reqs, "iso_s": list(iso_ns * 1e-9), "iso_span_s": iso_span,
                                     "footprints": [serve_footprint(q) for q in reqs], "budget": budget,
                                     "bound": args.bound, "slots": slots,
                                     "latency_ms_p50": run["latency_ms_p50"], "latency_ms_p99": run["latency_ms_p99"]})
        if lam != 1000.0:
            continue
        duty = 25
        bg_ops, bg_ws, bg = background_load(ctx, ctx.device, duty)
        for policy in ("naive", "sensitivity"):
            q0 = ctx.queue_stats()
            t0 = time.perf_counter()
            res, rep = ctx.serve_loaded(reqs, "hbm", 1.0, ws=bg_ws, policy=policy, bound=args.bound,
                                        hbm_budget=budget, slots=slots, profiles=profiles, background=bg,
                                        duty=duty, deadline_ms=int(1000 * (60 + 20 * seconds)), **bg_ops)
            wall = time.perf_counter() - t0
            q1 = ctx.queue_stats()
            run = {"rate_per_s": lam, "seconds": seconds, "policy": policy, "requests": len(reqs)}
            run.update(_serving_stats(res, reqs, iso_ns, args.bound))
            run.update({"slowdown_over": "every request (service in the mix / service alone on an idle device)",
                        "results_equal_isolated": all(r["checksum_bits"] == i["checksum_bits"]
                                                      for r, i in zip(res, iso)),
                        "background": {"stressor": "hbm triad, every CU", "duty_pct": duty,
                                       "load": round(bg["press"]["hbm"], 4),
                                       "predicted_slowdown_beside_it_alone":
                                           {k: round(coloc.predict_slowdown(profiles, k, [bg]), 3) for k in profiles},
                                       "stressor_gb_s": round(rep.achieved / 1e9, 1),
                                       "slot_queue_check": {k: q1[k] - q0[k] for k in q1}},
                        "wall_s": round(wall, 1)})
            summary["runs"].append(run)
            log(f"serve {lam}/s {policy} under the background: {run}")
            if keep_host:
                host["runs"].append({"rate": lam, "policy": policy, "reqs": reqs, "iso_s": list(iso_ns * 1e-9), "iso_span_s": iso_span,
                                     "footprints": [serve_footprint(q) for q in reqs], "budget": budget,
                                     "bound": args.bound, "slots": slots, "background": bg,
                                     "latency_ms_p50": run["latency_ms_p50"], "latency_ms_p99": run["latency_ms_p99"]})
        del bg_ops, bg_ws
    summary["profiles"] = profiles
    return summary, host


def serve_footprint(q):
    """Bytes a request holds in the loop's arena (rounded as the loop rounds)."""
    al = lambda b: (b + 255) // 256 * 256
    if q["kind"] == "triad":
        return 3 * al(q["n"] * 4)
    if q["kind"] == "gemm":
        e = {"f32": 4, "bf16": 2}[q.get("dtype", "bf16")]
        stage = 0 if q.get("dtype") == "f32" else max(q["m"], q["n"]) * q["k"] * 4
        return al(q["m"] * q["k"] * e) + al(q["n"] * q["k"] * e) + al(q["m"] * q["n"] * 4) + al(stage)
    return al(q["n"] * q["k"] * 2) + al(q["k"] * 2) + al(q["n"] * 4) + al(max(q["n"] * q["k"], q["k"]) * 4)


def run_suite(args):
    import torch
    from paper_2501_16909_amd import coloc
    dev = torch.device("cuda:0")
    ctx = coloc.Context(0)
    t_start = time.perf_counter()
    suite = Suite(ctx, dev)
    log("setup done")
    warm = {}
    for i in range(args.warmup):
        suite.step(warm, args.stressor_warmup)
    acc = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        suite.step(acc, args.stressor_warmup)
        log(f"step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stress = {}
    for name, _, unit, scale in suite.items:
        a = acc[name]
        rate = float(np.mean(a["rates"]))
        pct = a["pct"][0]
        stress[name] = {"achieved": round(rate / scale, 3), "unit": unit,
                        "pct_of_peak": None if pct is None else round(float(np.mean(a["pct"])), 1),
                        "kernel_ms": round(float(np.mean(a["kernel_ns"])) / 1e6, 4)}
    pairs = {}
    for placement in ("shared", "disjoint"):
        cells = acc["pair_" + placement]
        pairs[placement] = {"slowdown": round(float(np.median([c["slowdown"] for c in cells])), 3),
                            "t_alone_us": round(float(np.median([c["t_alone_ns"] for c in cells])) / 1e3, 2),
                            "t_coloc_us": round(float(np.median([c["t_col_ns"] for c in cells])) / 1e3, 2),
                            "output_equal": all(c["output_equal"] for c in cells),
                            "window_covered": all(c["window_covered"] for c in cells),
                            "stressor_cus": cells[0]["ncu"]}
    hbm = acc["hbm"]
    t_ns = float(np.mean(hbm["kernel_ns"]))
    achieved = hbm["units"] / t_ns  # GB/s (bytes per ns)
    traffic = hbm_traffic()
    line = {
        "metric": METRIC,
        "value": round(achieved, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (SplitMix64 counter-form uniform [-1,1) / uint32 words / random cycle)",
        "config": {"workload": "stressor suite standalone: HBM triad FP32 N=2^30 (and its "
                               "read-only, copy and write-only mixes); L2 2 MiB; "
                               "Infinity Cache 128 MiB (read, also at 32 waves/CU, and write-only); vL1D 16 KiB; LDS 64 KiB/WG copy "
                               "(L2 and LDS also at 32 waves/CU) and load-only (also at 32 waves/CU); FP32 FMA and FP64 multiply chains 4096; "
                               "MFMA FP32/BF16/FP8; uint32 chase over 2^24 cycle; 10^6 empty "
                               "64-thread WGs; plus colocated triad pair N=2^22",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": 8000.0, "unit": "GB/s",
                     "frac": round(achieved / 8000.0, 4),
                     "traffic": traffic,
                     "kernel": "stream_stressor<1u, true, 4, true>: triad mix, fixed work "
                               "(12 B per element, N=2^30, one pass per launch)"},
        "stressors": stress,
        "colocated_triad_pair": pairs,
    }
    log(f"suite: {wall:.1f} s timed; hbm {achieved:.0f} GB/s")
    host_arrays = None
    if not args.no_cpu_baseline:      # the headline arrays, for the oracle's triad on the host
        host_arrays = (suite.hb.cpu().numpy(), suite.hc.cpu().numpy())
    prec_host = serve_host = sens_host = None
    if not args.quick:
        ws = suite.ws
        del suite
        torch.cuda.empty_cache()
        line["sensitivity"], sens_host = sensitivity_block(ctx, dev, args.suite_reps, ws, not args.no_cpu_baseline)
        log(f"sensitivity block done at {time.perf_counter() - t_start:.0f} s")
        line["precision"], prec_host = precision_block(ctx, dev, not args.no_cpu_baseline)
        log(f"precision block done at {time.perf_counter() - t_start:.0f} s")
        line["serving"], serve_host = serving_block(ctx, args, not args.no_cpu_baseline)
        log(f"serving block done at {time.perf_counter() - t_start:.0f} s")
    ctx.close()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(host_arrays, prec_host, serve_host, sens_host)
        log(f"cpu baseline done at {time.perf_counter() - t_start:.0f} s")
    print(json.dumps(line), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(line, f)



# --------------------------------------------------------------------------
# Sensitivity sweep, precision and serving workloads (their own JSON lines)
# --------------------------------------------------------------------------
INTENSITIES = [0.0, 0.25, 0.5, 0.75, 1.0]


def stressor_operands(dev):
    """Operands for every stressor at the sweep's sizes."""
    import torch
    import synth
    T = lambda x: torch.from_numpy(np.require(x, requirements=["C", "W"])).to(dev)
    n = 1 << 28
    hb = torch.empty(n, dtype=torch.float32, device=dev)
    hc, ha = torch.empty_like(hb), torch.empty_like(hb)
    synth.device_fill_uniform_f32(hb.data_ptr(), n, synth.seed_for(2, synth.BUF_B))
    synth.device_fill_uniform_f32(hc.data_ptr(), n, synth.seed_for(2, synth.BUF_C))
    l2 = torch.empty(1 << 19, dtype=torch.int32, device=dev)
    l1 = torch.empty(1 << 12, dtype=torch.int32, device=dev)
    for t, k in ((l2, 0), (l1, 2)):
        synth.device_fill_u32(t.data_ptr(), t.numel(), synth.seed_for(2, synth.BUF_CACHE) + k)
    nm = 1 << 24   # Infinity Cache: two 64 MiB arrays read (16 MiB per XCD slot)
    mb = torch.empty(nm, dtype=torch.float32, device=dev)
    mc = torch.empty_like(mb)
    synth.device_fill_uniform_f32(mb.data_ptr(), nm, synth.seed_for(2, synth.BUF_CACHE) + 1)
    synth.device_fill_uniform_f32(mc.data_ptr(), nm, synth.seed_for(2, synth.BUF_CACHE) + 3)
    win = T(synth.u32(synth.seed_for(2, synth.BUF_LDS), 8192).view(np.int32))
    valu = torch.empty(256 * 4 * 256 * 8, dtype=torch.float32, device=dev)
    mf = {"f32": (np.ones((32, 2), np.float32), np.ones((2, 32), np.float32)),
          "bf16": (np.full((32, 16), 0x3F80, np.int16), np.full((16, 32), 0x3F80, np.int16)),
          "fp8": (np.full((32, 64), 0x38, np.uint8), np.full((64, 32), 0x38, np.uint8))}
    mf = {k: (T(a), T(b)) for k, (a, b) in mf.items()}
    mout = torch.empty(256 * 2 * 4 * 4 * 1024, dtype=torch.float32, device=dev)
    chase = T(synth.random_cycle_u32(synth.seed_for(2, synth.BUF_CHASE), 1 << 24).view(np.int32))
    cend = torch.empty(256 * 256 * 4, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    return {
        "hbm": dict(src0=hb, src1=hc, dst=ha, n=n),
        "l2": dict(src0=l2, n=1 << 19),
        "mall": dict(src0=mb, src1=mc, n=nm),
        "vl1d": dict(src0=l1, n=1 << 12),
        "lds": dict(src0=win),
        "valu_f32": dict(dst=valu, fa=1 - 2 ** -12, fb=2 ** -12),
        "mfma_f32": dict(src0=mf["f32"][0], src1=mf["f32"][1], dst=mout),
        "mfma_bf16": dict(src0=mf["bf16"][0], src1=mf["bf16"][1], dst=mout),
        "mfma_fp8": dict(src0=mf["fp8"][0], src1=mf["fp8"][1], dst=mout),
        "ptrchase": dict(src0=chase, n=1 << 24, dst=cend),
        "dispatch": dict(iters=100000),
        "occupancy": dict(),
    }


def sweep_victims(ctx, dev):
    import torch
    import synth
    m = 4096
    a = torch.empty(m * m, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    a.copy_(torch.from_numpy(synth.normal_f32(synth.seed_for(2, synth.BUF_GEMM_A), m * m)))
    b.copy_(torch.from_numpy(synth.normal_f32(synth.seed_for(2, synth.BUF_GEMM_B), m * m)))
    qa, _ = ctx.quantize(a, "bf16")
    qb, _ = ctx.quantize(b, "bf16")
    c = torch.empty((m, m), dtype=torch.float32, device=dev)
    gemm = ctx.gemm_desc(qa, qb, c, "bf16", m, m, m)
    n = 8192
    w = torch.from_numpy(synth.normal_f32(synth.seed_for(2, synth.BUF_GEMV_W), n * n, sigma=0.02)).to(dev)
    x = torch.from_numpy(synth.normal_f32(synth.seed_for(2, synth.BUF_GEMV_X), n)).to(dev)
    qw, _ = ctx.quantize(w, "bf16")
    qx, _ = ctx.quantize(x, "bf16")
    w3 = qw.repeat(3)          # three identical weight copies, rotated over runs (384 MiB)
    y = torch.empty(n, dtype=torch.float32, device=dev)
    gemv = ctx.gemv_desc(w3, qx, y, n, n, copies=3)
    t = 1 << 24
    tb = torch.empty(t, dtype=torch.float32, device=dev)
    tc, ta = torch.empty_like(tb), torch.empty_like(tb)
    synth.device_fill_uniform_f32(tb.data_ptr(), t, synth.seed_for(2, synth.BUF_B2))
    synth.device_fill_uniform_f32(tc.data_ptr(), t, synth.seed_for(2, synth.BUF_C2))
    triad = ctx.triad_desc(tb, tc, ta, passes=2)
    del a, b, w
    return {"gemm_bf16_4096": gemm, "gemv_bf16_8192": gemv, "triad_f32_2e24": triad}


def run_sweep(args):
    import torch
    from paper_2501_16909_amd import coloc
    dev = torch.device("cuda:0")
    ctx = coloc.Context(0)
    ops = stressor_operands(dev)
    victims = sweep_victims(ctx, dev)
    # rows: every stressor in its default shape, plus the pipe stressors
    # with one wave per SIMD (a 256-thread work-group per CU), which leave
    # issue slots to co-resident victims
    rows = [(r, r, ops[r]) for r in ops]
    for r in ("valu_f32", "mfma_bf16"):
        rows.append((r + "_1wave", r, dict(ops[r], wg_per_cu=1, threads=256)))
    res = [r for _, r, _ in rows]
    ws = torch.empty(WS_BYTES, dtype=torch.uint8, device=dev)
    out = {"metric": "victim slowdown per resource vs intensity", "config": {
        "workload": "sensitivity sweep: BF16 GEMM 4096^3 and BF16 GEMV 8192^2 (3 rotating weight "
                    "copies) x 12 stressors x CU intensity 0/25/50/75/100%", "reps": args.reps},
        "intensities": INTENSITIES, "tables": {}}
    t0 = time.perf_counter()
    for placement in ("shared", "disjoint"):
        for vname, d in victims.items():
            tab = {}
            for i, (r, rr, o) in enumerate(rows):
                # one call per stressor row: each ends with a log line
                row = ctx.measure_sensitivity(d, [rr], [o], INTENSITIES, reps=args.reps, warmups=3,
                                              placement=placement, ws=ws, deadline_ms=args.deadline_ms)
                log(f"{vname} {placement} {r}: {[round(c['slowdown'], 3) for c in row]}")
                nan = lambda v: v != v
                tab[r] = {"slowdown": [None if nan(c["slowdown"]) else round(c["slowdown"], 3) for c in row],
                          "p90": [None if nan(c["slowdown_p90"]) else round(c["slowdown_p90"], 3) for c in row],
                          "ci95": [None if nan(c["slowdown_ci_lo"]) else
                                   [round(c["slowdown_ci_lo"], 3), round(c["slowdown_ci_hi"], 3)] for c in row],
                          "stressor_pct_peak": [round(c["stressor_pct_peak"], 1) for c in row],
                          # a stressor that hit its deadline outlived the victim's
                          # starvation: the slowdown is then a lower bound
                          "starved": [bool(c["timed_out"]) for c in row],
                          "valid": [bool(c["window_covered"] and c["output_equal"] and not c["queue_unresolved"])
                                    and not nan(c["slowdown"])
                                    for c in row],
                          "t_alone_us": [None if nan(c["t_alone_ns"]) else round(c["t_alone_ns"] / 1e3, 2) for c in row]}
            out["tables"][f"{vname}/{placement}"] = tab
            log(f"{vname} {placement}: " + ", ".join(f"{r}={tab[r]['slowdown'][-2]}" for r in tab))
    out["seconds"] = round(time.perf_counter() - t0, 1)
    out["queue_pair_check"] = ctx.queue_stats()
    ctx.close()
    print(json.dumps(out), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(out, f)


def run_hbm_mix(args):
    """Victim slowdown against the HBM stressor in each traffic mix (triad,
    read-only, copy, write-only) at CU intensity 0/25/50/75/100 %, with the
    stressor's own bandwidth in each cell: how much of a memory-bound
    co-runner's harm depends on its read/write proportion."""
    import torch
    from paper_2501_16909_amd import coloc
    dev = torch.device("cuda:0")
    ctx = coloc.Context(0)
    h = stressor_operands(dev)["hbm"]
    victims = sweep_victims(ctx, dev)
    mixes = {"triad": dict(src0=h["src0"], src1=h["src1"], dst=h["dst"]),
             "read": dict(src0=h["src0"], src1=h["src1"]),
             "copy": dict(src0=h["src0"], dst=h["dst"]),
             "write": dict(dst=h["dst"])}
    opts = [dict(o, n=h["n"], knob=coloc.HBM_MIX[m]) for m, o in mixes.items()]
    ws = torch.empty(WS_BYTES, dtype=torch.uint8, device=dev)
    out = {"metric": "victim slowdown vs HBM traffic mix and intensity", "config": {
        "workload": "victims of the sensitivity sweep x HBM stressor over 2^28-element FP32 arrays "
                    "in four read/write mixes x CU intensity 0/25/50/75/100%", "reps": args.reps},
        "intensities": INTENSITIES, "tables": {}}
    t0 = time.perf_counter()
    for placement in ("shared", "disjoint"):
        for vname, d in victims.items():
            cells = ctx.measure_sensitivity(d, ["hbm"] * len(mixes), opts, INTENSITIES, reps=args.reps,
                                            warmups=3, placement=placement, ws=ws,
                                            deadline_ms=args.deadline_ms)
            tab = {}
            for i, m in enumerate(mixes):
                row = cells[i * len(INTENSITIES):(i + 1) * len(INTENSITIES)]
                nan = lambda v: v != v
                tab[m] = {"slowdown": [None if nan(c["slowdown"]) else round(c["slowdown"], 3) for c in row],
                          "stressor_gbs": [round(c["stressor_achieved"] / 1e9, 1) for c in row],
                          "valid": [bool(c["window_covered"] and c["output_equal"] and not c["queue_unresolved"])
                                    and not nan(c["slowdown"])
                                    for c in row]}
            out["tables"][f"{vname}/{placement}"] = tab
            log(f"{vname} {placement}: " + ", ".join(f"{m}={tab[m]['slowdown'][-1]}" for m in tab))
    out["seconds"] = round(time.perf_counter() - t0, 1)
    out["queue_pair_check"] = ctx.queue_stats()
    ctx.close()
    _emit(out, args)


def run_precision(args):
    """GEMM M = N = K = 8192 in FP32, BF16 and FP8 (per-tensor scale) from
    N(0,1) inputs, FP32 accumulation: time and rate per dtype, the
    sensitivity row per dtype, and (CPU leg) the error against FP64 on 4096
    sampled entries: kernel error (FP64 product of the quantised inputs) and
    total error (FP64 product of the FP32 inputs), normalised by |A||B|^T,
    normwise, and over the dtype's bound."""
    import torch
    from paper_2501_16909_amd import coloc
    dev = torch.device("cuda:0")
    ctx = coloc.Context(0)
    summary, host = precision_block(ctx, dev, True)
    m = 8192
    ops = stressor_operands(dev)
    ws = torch.empty(WS_BYTES, dtype=torch.uint8, device=dev)
    out = {"metric": "GEMM error vs FP64 and sensitivity per dtype",
           "config": {"workload": "GEMM M=N=K=8192, inputs N(0,1), FP32 accumulate; FP8 e4m3 per-tensor scale",
                      "sample": "4096 fixed-seed entries"}, "dtypes": summary}
    import synth
    ha = synth.normal_f32(synth.seed_for(3, synth.BUF_GEMM_A), m * m).reshape(m, m)
    hb = synth.normal_f32(synth.seed_for(3, synth.BUF_GEMM_B), m * m).reshape(m, m)
    a, b = torch.from_numpy(ha).to(dev), torch.from_numpy(hb).to(dev)
    c = torch.empty((m, m), dtype=torch.float32, device=dev)
    for dt in ("f32", "bf16", "fp8"):
        if dt == "f32":
            qa, qb, sa, sb = a, b, 1.0, 1.0
        else:
            qa, sa = ctx.quantize(a, dt)
            qb, sb = ctx.quantize(b, dt)
        d = ctx.gemm_desc(qa, qb, c, dt, m, m, m, sa, sb)
        res = list(ops)
        cells = ctx.measure_sensitivity(d, res, [ops[r] for r in res], [0.0, 0.5, 1.0], reps=args.reps,
                                        warmups=1, ws=ws, deadline_ms=args.deadline_ms)
        summary[dt]["sensitivity"] = {r: [round(cells[i * 3 + j]["slowdown"], 3) for j in range(3)]
                                      for i, r in enumerate(res)}
        summary[dt]["sensitivity_intensities"] = [0.0, 0.5, 1.0]
        log(f"{dt}: sensitivity {summary[dt]['sensitivity']}")
    ctx.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = {"kind": "oracle", "precision": _cpu_precision_leg(host)}
    _emit(out, args)


def serve_trace(lam, seconds, seed):
    """Poisson arrivals; a third each of BF16 GEMM (n ~ log-U[512, 8192],
    multiple of 128), BF16 GEMV (n ~ log-U[4096, 16384], multiple of 8) and
    FP32 triad (N ~ log-U[2^20, 2^28])."""
    import synth
    w = synth.words(seed, 4 * int(lam * seconds * 2 + 16))
    u = ((w >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53
    reqs, t, i = [], 0.0, 0
    while True:
        t += -np.log(u[i]) / lam
        i += 1
        if t > seconds:
            break
        kind = int(u[i] * 3)
        i += 1
        x = u[i]
        i += 1
        if kind == 0:
            n = int(round(np.exp(np.log(512) + x * (np.log(8192) - np.log(512))) / 128)) * 128
            reqs.append({"arrival_s": t, "kind": "gemm", "dtype": "bf16", "m": n, "n": n, "k": n})
        elif kind == 1:
            n = int(round(np.exp(np.log(4096) + x * (np.log(16384) - np.log(4096))) / 8)) * 8
            reqs.append({"arrival_s": t, "kind": "gemv", "dtype": "bf16", "n": n, "k": n})
        else:
            n = int(np.exp(np.log(2.0 ** 20) + x * (np.log(2.0 ** 28) - np.log(2.0 ** 20))))
            reqs.append({"arrival_s": t, "kind": "triad", "n": n})
        reqs[-1]["seed"] = 900000 + 10 * len(reqs)
    return reqs


DUTIES = (10, 25, 50, 75, 100)
CURVE_DUTIES = (25, 50, 75, 100)   # with duty 0, the five points of a duty-axis curve


def equivalent_duty(frac, duty_rates, full):
    """The stressor duty (0..1) whose standalone rate is `frac` of the full
    rate: linear between the measured duty levels (duty_rates: percent ->
    rate), from rate 0 at duty 0; 1 at or beyond the top level's rate.  A
    co-runner's pressure on the duty axis is this equivalent intensity, so
    that it reads the victim's curve where the stressor matched its use."""
    ds = [0.0] + [d / 100.0 for d in sorted(duty_rates)]
    xs = [0.0]
    for d in sorted(duty_rates):       # rates rise with duty; keep the table increasing
        xs.append(max(duty_rates[d] / full, xs[-1] + 1e-9))
    return float(np.interp(frac, xs, ds))
# Write share of each request kind's compulsory HBM bytes: the GEMV reads its
# weights and writes one short vector, the triad writes one stream of three,
# the GEMM writes an FP32 C as large as its BF16 A and B together.
HBM_WRITE_FRAC = {"gemm": 0.5, "gemv": 0.0, "triad": 1.0 / 3.0}
# Working set of each request kind at the profiled sizes (GEMM 2048^3 BF16 in,
# FP32 out; GEMV 8192^2 BF16; triad three 2^24 FP32 arrays), against the
# 256 MB Infinity Cache: a co-runner that fits is served from it when it
# runs back to back, not from DRAM.
KIND_FOOTPRINT = {"gemm": 2 * 2048 * 2048 * 2 + 2048 * 2048 * 4, "gemv": 8192 * 8192 * 2 + 8192 * 6,
                  "triad": 3 * 4 * (1 << 24)}
MALL_BYTES = 256 * 10 ** 6


def serve_profiles(ctx, args, axis="cu", hbm_mix="triad", res=("hbm", "mfma_bf16", "lds")):
    """Sensitivity profiles of the three request kinds at representative
    sizes (GEMM BF16 2048^3, GEMV BF16 8192^2, triad N = 2^24): slowdown
    curves (shared placement) on the resources the kinds themselves load --
    HBM, BF16 matrix cores, LDS -- and the pressure each kind exerts there,
    from its standalone use of the unit against the matching stressor's
    standalone rate (as below, per axis).

    axis "cu": the stressor runs at full rate on a fraction x of the CUs;
    pressure is the use over the full rate.
    axis "duty": the stressor runs on every CU, active a fraction of the
    time; the curve's points are duty 0, 25, 50, 75 and 100 %, and a kind's
    pressure is the equivalent duty: the duty at which the stressor's
    standalone rate matches the kind's use (equivalent_duty).

    hbm_mix picks the HBM stressor's traffic mix ("triad" or "read"); res
    limits the resources profiled."""
    import torch
    import synth
    from paper_2501_16909_amd.coloc import HBM_MIX
    dev = ctx.device
    ops = stressor_operands(dev)
    if hbm_mix == "read":
        h = ops["hbm"]
        ops["hbm"] = dict(src0=h["src0"], src1=h["src1"], n=h["n"], knob=HBM_MIX["read"])
    res = list(res)
    ws = torch.empty(WS_BYTES, dtype=torch.uint8, device=dev)
    rates = {}
    duty_rates = {}
    fixed = {"hbm": dict(passes=1), "mfma_bf16": dict(iters=2048, passes=2), "lds": dict(passes=4),
             "mall": dict(passes=60)}

    def steady_rate(r, **kw):
        # median of three launches after an untimed one: a stressor's first
        # launch in a process can run 20 % slow, which would shift every
        # load measured against it
        run = lambda: ctx.stressor(r, 1.0, ws=ws, **ops[r], **fixed[r], **kw).stop()
        run()
        return float(np.median([(lambda rep: rep.units / (rep.kernel_ns * 1e-9))(run()) for _ in range(3)]))

    for r in res:
        rates[r] = steady_rate(r)
        if axis == "duty":
            duty_rates[r] = {duty: steady_rate(r, duty=duty) for duty in DUTIES}
            log(f"{r} duty rates (fraction of full): "
                + ", ".join(f"{k}%: {v / rates[r]:.3f}" for k, v in duty_rates[r].items()))
    g = 2048
    A = torch.from_numpy(synth.uniform_f32(11, g * g)).to(dev)
    B = torch.from_numpy(synth.uniform_f32(12, g * g)).to(dev)
    qa, _ = ctx.quantize(A, "bf16")
    qb, _ = ctx.quantize(B, "bf16")
    C = torch.empty((g, g), dtype=torch.float32, device=dev)
    n = 8192
    W = torch.from_numpy(synth.uniform_f32(13, n * n)).to(dev)
    X = torch.from_numpy(synth.uniform_f32(14, n)).to(dev)
    qw, _ = ctx.quantize(W, "bf16")
    qx, _ = ctx.quantize(X, "bf16")
    Y = torch.empty(n, dtype=torch.float32, device=dev)
    t = 1 << 24
    tb = torch.from_numpy(synth.uniform_f32(15, t)).to(dev)
    tc = torch.from_numpy(synth.uniform_f32(16, t)).to(dev)
    ta = torch.empty_like(tb)
    descs = {"gemm": ctx.gemm_desc(qa, qb, C, "bf16", g, g, g), "gemv": ctx.gemv_desc(qw, qx, Y, n, n),
             "triad": ctx.triad_desc(tb, tc, ta, passes=1)}
    # standalone use of each resource (algorithmic bytes / flops per run)
    gemm_lds = (g // 128) ** 2 * (g * 2 // 128) * (4 * 16384 + 32768)   # per stage: reads + writes
    use = {"gemm": {"mfma_bf16": 2.0 * g ** 3, "lds": gemm_lds, "hbm": 3.0 * 2 * g * g},
           "gemv": {"hbm": 2.0 * n * n}, "triad": {"hbm": 12.0 * t}}
    for u in use.values():    # the same bytes, priced against the Infinity-Cache stressor
        u["mall"] = u["hbm"]
    occ = {"gemm": min(1.0, (g // 128) ** 2 / (256 * 2)) * 8 / 32, "gemv": 1.0, "triad": 1.0}
    profiles = {}
    for kind, d in descs.items():
        t_alone = float(np.median([ctx.victim_run(d).time_ns for _ in range(5)])) * 1e-9
        sens = {}
        if axis == "cu":
            cells = ctx.measure_sensitivity(d, res, [ops[r] for r in res], INTENSITIES, reps=args.reps,
                                            warmups=2, ws=ws, deadline_ms=args.deadline_ms)
            for i, r in enumerate(res):
                row = cells[i * len(INTENSITIES):(i + 1) * len(INTENSITIES)]
                sens[r] = [float(c["slowdown"]) if c["slowdown"] == c["slowdown"] else 1.0 for c in row]
        else:
            # the curve's points: the stressor on every CU at duty 0, 25, 50,
            # 75 and 100 %
            sens = {r: [1.0] for r in res}
            for duty in CURVE_DUTIES:
                cells = ctx.measure_sensitivity(d, res, [dict(ops[r], duty=duty) for r in res], [1.0],
                                                reps=args.reps, warmups=2, ws=ws,
                                                deadline_ms=args.deadline_ms)
                for i, r in enumerate(res):
                    sens[r].append(float(cells[i]["slowdown"]))
        frac = {r: use[kind].get(r, 0.0) / t_alone / rates[r] for r in res}
        if axis == "cu":
            press = {r: min(1.0, frac[r]) for r in res}
        else:
            press = {r: equivalent_duty(frac[r], duty_rates[r], rates[r]) for r in res}
        profiles[kind] = {"sens": sens, "press": press, "occ": occ[kind],
                          "hbm_write_frac": HBM_WRITE_FRAC[kind]}
    return profiles


def run_serve(args):
    """Serving loop at several arrival rates, naive versus sensitivity-aware
    admission; latency p50/p99, throughput, and slowdown of service time
    against the same request served alone (sampled)."""
    import torch
    from paper_2501_16909_amd import coloc
    ctx = coloc.Context(0)
    if args.profiles and os.path.exists(args.profiles):
        with open(args.profiles) as f:
            profiles = json.load(f)
    else:
        profiles = median_profiles([serve_profiles(ctx, args, axis=args.profile_axis)
                                    for _ in range(max(1, args.profile_runs))])
        log("profiles: " + json.dumps(profiles))
    out = {"metric": "serving latency p50/p99 and throughput, naive vs occupancy-based vs sensitivity-aware admission",
           "config": {"workload": "Poisson arrivals, 1/3 each BF16 GEMM n~logU[512,8192], BF16 GEMV "
                                  "n~logU[4096,16384], FP32 triad N~logU[2^20,2^28]",
                      "seconds": args.seconds, "slots": 4, "hbm_budget_gib": 32,
                      "profile_axis": args.profile_axis, "profile_runs": max(1, args.profile_runs)},
           "runs": []}
    iso_cache = {}
    for lam in args.rates:
        reqs = serve_trace(lam, args.seconds, 31337 + int(lam))
        for policy in (["naive", "usher", "sensitivity"] if profiles else ["naive"]):
            t0 = time.perf_counter()
            res = ctx.serve(reqs, policy=policy, bound=args.bound, hbm_budget=32 << 30, slots=4,
                            profiles=profiles)
            wall = time.perf_counter() - t0
            lat = np.array([r["end_s"] - r["arrival_s"] for r in res])
            svc = np.array([r["service_ns"] for r in res])
            # isolated service time for a fixed sample of requests
            sample = list(range(0, len(reqs), max(1, len(reqs) // 40)))
            ratios = []
            for i in sample:
                key = json.dumps({k: v for k, v in reqs[i].items() if k != "arrival_s"}, sort_keys=True)
                if key not in iso_cache:
                    iso = ctx.serve([dict(reqs[i], arrival_s=0.0)], policy="naive", hbm_budget=32 << 30, slots=1)[0]
                    iso_cache[key] = iso
                iso = iso_cache[key]
                assert iso["checksum_bits"] == res[i]["checksum_bits"], "result differs alone vs in the mix"
                ratios.append(res[i]["service_ns"] / iso["service_ns"])
            out["runs"].append({"rate_per_s": lam, "policy": policy, "requests": len(reqs),
                                "latency_ms_p50": round(float(np.percentile(lat, 50)) * 1e3, 3),
                                "latency_ms_p99": round(float(np.percentile(lat, 99)) * 1e3, 3),
                                "throughput_req_s": round(len(reqs) / max(r["end_s"] for r in res), 1),
                                "service_ms_mean": round(float(svc.mean()) / 1e6, 4),
                                "slowdown_p50": round(float(np.percentile(ratios, 50)), 3),
                                "slowdown_p99": round(float(np.percentile(ratios, 99)), 3),
                                "results_equal_isolated": True, "wall_s": round(wall, 2)})
            log(json.dumps(out["runs"][-1]))
    ctx.close()
    print(json.dumps(out), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(out, f)



def _serving_stats(res, reqs, iso_ns, bound):
    lat = np.array([r["end_s"] - r["arrival_s"] for r in res])
    slow = np.array([r["service_ns"] for r in res]) / iso_ns
    horizon = max(r["end_s"] for r in res)
    kinds = np.array([q["kind"] for q in reqs])
    return {"slowdown_p50_by_kind": {k: round(float(np.median(slow[kinds == k])), 3)
                                     for k in ("gemm", "gemv", "triad") if np.any(kinds == k)},"latency_ms_p50": round(float(np.percentile(lat, 50)) * 1e3, 3),
            "latency_ms_p99": round(float(np.percentile(lat, 99)) * 1e3, 3),
            "throughput_req_s": round(len(reqs) / horizon, 1),
            "slowdown_p50": round(float(np.percentile(slow, 50)), 3),
            "slowdown_p99": round(float(np.percentile(slow, 99)), 3),
            "over_bound_frac": round(float(np.mean(slow > bound)), 4),
            "mean_in_service": round(float(sum(r["end_s"] - r["admit_s"] for r in res)) / horizon, 3)}


def run_serve_background(args):
    """Serving on a loaded device: an HBM triad stressor on every CU at duty
    --duty (traffic mix --background-mix) runs through each serving run (serve_run_background), so that the
    admission rule has to decide against a constant background load; naive,
    occupancy-based (usher) and sensitivity-aware admission (duty-axis profiles with
    read/write-aware HBM pricing, the stressor's own measured load as the
    rule's background), and the same traces without the stressor.
    Slowdowns are over every request, against the request served alone on
    an idle device; every result must equal its isolated one bit for bit."""
    import torch
    from paper_2501_16909_amd import coloc
    ctx = coloc.Context(0)
    dev = ctx.device
    profiles = library_profiles(serve_profiles(ctx, args, axis="duty"),
                                serve_profiles(ctx, args, axis="duty", hbm_mix="read", res=("hbm",)))
    ops, ws, bg = background_load(ctx, dev, args.duty, args.background_mix)
    press = bg["press"]["hbm"]
    alone_bg = {k: round(coloc.predict_slowdown(profiles, k, [bg]), 3) for k in profiles}
    log(f"background: HBM {args.background_mix} stressor, duty {args.duty} %: load {press:.3f} of the "
        f"triad's full rate; predicted slowdown beside it alone: {alone_bg}")
    budget, slots = 32 << 30, 4
    out = {"metric": "serving latency p50/p99, throughput and slowdown under a background HBM stressor, "
                     "naive vs occupancy-based vs sensitivity-aware admission",
           "config": {"workload": "Poisson arrivals, 1/3 each BF16 GEMM n~logU[512,8192], BF16 GEMV "
                                  "n~logU[4096,16384], FP32 triad N~logU[2^20,2^28]",
                      "seconds": args.seconds, "slots": slots, "hbm_budget_gib": budget >> 30,
                      "bound": args.bound, "profile_axis": "duty", "hbm_pricing": "read/write-aware",
                      "background": {"resource": "hbm", "mix": args.background_mix, "intensity": 1.0,
                                     "duty_pct": args.duty, "load": round(press, 4),
                                     "load_read": round(bg.get("press_hbm_read", 0.0), 4), "occ": 0.25,
                                     "predicted_slowdown_beside_it_alone": alone_bg}},
           "runs": [], "profiles": profiles}
    for lam in args.rates:
        reqs = serve_trace(lam, args.seconds, 31337 + int(lam))
        iso = ctx.serve([dict(r, arrival_s=0.0) for r in reqs], policy="naive", hbm_budget=budget, slots=1)
        iso_ns = np.array([o["service_ns"] for o in iso])
        for loaded in (False, True):
            for policy in ("naive", "usher", "sensitivity"):
                log(f"serve {lam}/s {policy}, background {'on' if loaded else 'off'}: {len(reqs)} requests")
                t0 = time.perf_counter()
                rep = None
                if loaded:
                    q0 = ctx.queue_stats()
                    res, rep = ctx.serve_loaded(reqs, "hbm", 1.0, ws=ws, policy=policy, bound=args.bound,
                                                hbm_budget=budget, slots=slots, profiles=profiles, background=bg,
                                                duty=args.duty, deadline_ms=int(1000 * (60 + 20 * args.seconds)),
                                                **ops)
                else:
                    res = ctx.serve(reqs, policy=policy, bound=args.bound, hbm_budget=budget, slots=slots,
                                    profiles=profiles)
                wall = time.perf_counter() - t0
                run = {"rate_per_s": lam, "policy": policy, "background": loaded, "requests": len(reqs)}
                run.update(_serving_stats(res, reqs, iso_ns, args.bound))
                run["results_equal_isolated"] = all(r["checksum_bits"] == i["checksum_bits"]
                                                    for r, i in zip(res, iso))
                if rep is not None:
                    q1 = ctx.queue_stats()
                    run["slot_queue_check"] = {k: q1[k] - q0[k] for k in q1}
                    run["stressor_gb_s"] = round(rep.achieved / 1e9, 1)
                    run["stressor_window_s"] = round(rep.window_ns * 1e-9, 3)
                run["wall_s"] = round(wall, 2)
                out["runs"].append(run)
                log(json.dumps(run))
                assert run["results_equal_isolated"], "a served result differs from its isolated run"
    ctx.close()
    print(json.dumps(out), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(out, f)

# --------------------------------------------------------------------------
# The paper's individual experiments, on MI355X
# --------------------------------------------------------------------------
def _gemv_victim(ctx, dev, n=8192, copies=3):
    import torch
    import synth
    w = torch.from_numpy(synth.normal_f32(synth.seed_for(2, synth.BUF_GEMV_W), n * n, sigma=0.02)).to(dev)
    x = torch.from_numpy(synth.normal_f32(synth.seed_for(2, synth.BUF_GEMV_X), n)).to(dev)
    qw, _ = ctx.quantize(w, "bf16")
    qx, _ = ctx.quantize(x, "bf16")
    y = torch.empty(n, dtype=torch.float32, device=dev)
    return ctx.gemv_desc(qw.repeat(copies), qx, y, n, n, copies=copies)


def _gemm_victim(ctx, dev, n):
    import torch
    import synth
    a = torch.from_numpy(synth.normal_f32(synth.seed_for(2, synth.BUF_GEMM_A), n * n)).to(dev)
    b = torch.from_numpy(synth.normal_f32(synth.seed_for(2, synth.BUF_GEMM_B), n * n)).to(dev)
    qa, _ = ctx.quantize(a, "bf16")
    qb, _ = ctx.quantize(b, "bf16")
    c = torch.empty((n, n), dtype=torch.float32, device=dev)
    return ctx.gemm_desc(qa, qb, c, "bf16", n, n, n)


def _cell(c):
    nan = lambda v: v != v
    return {"slowdown": None if nan(c["slowdown"]) else round(c["slowdown"], 3),
            "p10": None if nan(c["slowdown_p10"]) else round(c["slowdown_p10"], 3),
            "p90": None if nan(c["slowdown_p90"]) else round(c["slowdown_p90"], 3),
            "t_alone_us": None if nan(c["t_alone_ns"]) else round(c["t_alone_ns"] / 1e3, 2),
            "stressor_pct_peak": round(c["stressor_pct_peak"], 1),
            "valid": bool(c["window_covered"] and c["output_equal"]), "starved": bool(c["timed_out"])}


def run_pollution(args):
    """Cache pollution (Section 4.3, Figure 3 analog): two triad instances on
    disjoint halves of the CUs, data size per instance swept across the
    per-XCD L2 (4 MB) and the Infinity Cache (256 MB); slowdown of one."""
    import torch
    import synth
    from paper_2501_16909_amd import coloc
    ctx = coloc.Context(0)
    dev = ctx.device
    ws = torch.empty(WS_BYTES, dtype=torch.uint8, device=dev)
    rows = []
    for mib in (0.75, 1.5, 3, 6, 12, 24, 48, 96, 192, 384, 768, 1536):
        n = int(mib * (1 << 20) / 12) // 1024 * 1024
        bufs = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(6)]
        for i, t in enumerate(bufs):
            synth.device_fill_uniform_f32(t.data_ptr(), n, synth.seed_for(5, i))
        torch.cuda.synchronize()
        passes = max(1, int(300e-6 * 4e12 / (12 * n)))    # >= ~0.3 ms per victim run
        d = ctx.triad_desc(bufs[0], bufs[1], bufs[2], passes=passes, in_kernel=True)   # re-reads hit the caches
        so = [dict(src0=bufs[3], src1=bufs[4], dst=bufs[5], n=n, vec=1)]   # cached accesses, as the victim
        cell = ctx.measure_sensitivity(d, ["hbm"], so, [0.5], reps=args.reps, warmups=2, placement="disjoint",
                                       ws=ws, deadline_ms=args.deadline_ms)[0]
        r = _cell(cell)
        r.update({"mib_per_instance": mib, "n": n, "victim_passes": passes,
                  "victim_gbs_alone": round(12.0 * n * passes / cell["t_alone_ns"], 1)})
        rows.append(r)
        log(json.dumps(r))
        del bufs
        torch.cuda.empty_cache()
    out = {"metric": "slowdown vs data size per instance (cache pollution)",
           "config": {"workload": "two FP32 triads on disjoint CU halves (128 + 128 CUs), per-instance data "
                                  "= 3 arrays; victim timed, stressor persistent"}, "rows": rows}
    ctx.close()
    _emit(out, args)


def run_bandwidth(args):
    """L2/memory-bandwidth partition (Section 4.3, Table 1 analog): GEMV
    victim (BF16 8192^2, three rotated weight copies) on half the CUs, HBM
    stressor on the other half with 0..4 work-groups per CU."""
    import torch
    from paper_2501_16909_amd import coloc
    ctx = coloc.Context(0)
    dev = ctx.device
    ops = stressor_operands(dev)
    d = _gemv_victim(ctx, dev)
    ws = torch.empty(WS_BYTES, dtype=torch.uint8, device=dev)
    rows = []
    for wg in (0, 1, 2, 3, 4):
        if wg == 0:
            cell = ctx.measure_sensitivity(d, ["hbm"], [ops["hbm"]], [0.0], reps=args.reps, warmups=2,
                                           placement="disjoint", ws=ws)[0]
            cell_half = ctx.measure_sensitivity(d, ["hbm"], [ops["hbm"]], [0.5], reps=1, warmups=1,
                                                placement="disjoint", ws=ws)[0]
            r = _cell(cell)
            r["t_alone_half_us"] = round(cell_half["t_alone_ns"] / 1e3, 2)
        else:
            o = dict(ops["hbm"], wg_per_cu=wg)
            r = _cell(ctx.measure_sensitivity(d, ["hbm"], [o], [0.5], reps=args.reps, warmups=2,
                                              placement="disjoint", ws=ws, deadline_ms=args.deadline_ms)[0])
        r["stressor_wg_per_cu"] = wg
        r["stressor_workgroups"] = wg * 128
        rows.append(r)
        log(json.dumps(r))
    out = {"metric": "GEMV slowdown vs stressor work-groups on disjoint CUs (bandwidth partition)",
           "config": {"workload": "BF16 GEMV 8192^2 x 3 copies on 128 CUs; HBM triad stressor (N=2^28) on "
                                  "the other 128 CUs"}, "rows": rows}
    ctx.close()
    _emit(out, args)


def run_ilp(args):
    """Issue pressure (Section 4.4.2, Table 2 analog): FP32 FMA stressor with
    one 256-thread work-group per CU (one wave per SIMD) and ILP 1/2/4/8,
    on the same CUs as a GEMV and a triad victim."""
    import torch
    from paper_2501_16909_amd import coloc
    ctx = coloc.Context(0)
    dev = ctx.device
    ops = stressor_operands(dev)
    ws = torch.empty(WS_BYTES, dtype=torch.uint8, device=dev)
    victims = {"gemv_bf16_8192": _gemv_victim(ctx, dev)}
    import synth
    n = 1 << 24
    tb = torch.empty(n, dtype=torch.float32, device=dev)
    tc, ta = torch.empty_like(tb), torch.empty_like(tb)
    synth.device_fill_uniform_f32(tb.data_ptr(), n, 1)
    synth.device_fill_uniform_f32(tc.data_ptr(), n, 2)
    victims["triad_f32_2e24"] = ctx.triad_desc(tb, tc, ta, passes=2)
    out = {"metric": "victim slowdown vs VALU stressor ILP (issue pressure)",
           "config": {"workload": "FP32 FMA chains, 256 WGs x 256 threads (one wave per SIMD), ILP S1..S4 = "
                                  "1/2/4/8, same CUs as the victim"}, "rows": []}
    for ilp in (1, 2, 4, 8):
        o = dict(ops["valu_f32"], knob=ilp, wg_per_cu=1)
        rep = ctx.stressor("valu_f32", 1.0, ws=ws, iters=4096, passes=8, **o).stop()
        rate = rep.units / (rep.kernel_ns * 1e-9)
        # wave instructions per cycle per CU: FMAs / 64 lanes / (CUs x clock)
        ipc = rate / 2 / 64 / (256 * ctx.info.clock_khz * 1e3)
        row = {"ilp": ilp, "stressor_tflops": round(rate / 1e12, 2), "stressor_valu_ipc_per_cu": round(ipc, 3)}
        for vname, d in victims.items():
            c = ctx.measure_sensitivity(d, ["valu_f32"], [o], [1.0], reps=args.reps, warmups=2, ws=ws,
                                        deadline_ms=args.deadline_ms)[0]
            row[vname] = _cell(c)
        out["rows"].append(row)
        log(json.dumps(row))
    ctx.close()
    _emit(out, args)


def run_pairs(args):
    """Pipeline interference (Section 4.4.3, Table 3 analog) with two FP64
    multiply kernels of ILP 1/2/4/8, and the Pitfall-1 analog (Section 3):
    two FP32 FMA kernels with one wave per SIMD each."""
    import torch
    from paper_2501_16909_amd import coloc
    ctx1, ctx2 = coloc.Context(0), coloc.Context(0)
    dev = ctx1.device
    ws1 = torch.empty(WS_BYTES, dtype=torch.uint8, device=dev)
    ws2 = torch.empty_like(ws1)
    out64 = [torch.empty(256 * 256 * 8, dtype=torch.float64, device=dev) for _ in range(2)]
    out = {"metric": "seq/col speedup of two identical compute kernels",
           "config": {"workload": "each kernel 256 WGs x 256 threads (one wave per SIMD), all CUs, "
                                  "two hardware queues"}, "fp64_mul": [], "fp32_fma": []}
    for ilp in (1, 2, 4, 8):
        # both kernels write their own output buffer
        o = dict(knob=ilp, wg_per_cu=1, iters=4096, passes=16, fa=1 - 2 ** -20)
        r1 = ctx1.stressor("valu_f64", 1.0, ws=ws1, dst=out64[0], **o).stop()
        r2 = ctx2.stressor("valu_f64", 1.0, ws=ws2, dst=out64[1], **o).stop()
        seq = r1.window_ns + r2.window_ns
        s1 = ctx1.stressor("valu_f64", 1.0, ws=ws1, dst=out64[0], **o)
        s2 = ctx2.stressor("valu_f64", 1.0, ws=ws2, dst=out64[1], **o)
        a, b = s1.stop(), s2.stop()
        col_ns = (max(a.t_last_end, b.t_last_end) - min(a.t_first_start, b.t_first_start)) * 1e6 / ctx1.info.wall_clock_khz
        row = {"ilp": ilp, "fp64_pipe_util_alone_pct": round(r1.pct_of_peak, 1),
               "seq_ms": round(seq / 1e6, 4), "col_ms": round(col_ns / 1e6, 4),
               "speedup_seq_over_col": round(seq / col_ns, 3)}
        out["fp64_mul"].append(row)
        log(json.dumps(row))
    out32 = [torch.empty(256 * 256 * 8, dtype=torch.float32, device=dev) for _ in range(2)]
    for ilp in (1, 8):
        o = dict(knob=ilp, wg_per_cu=1, iters=4096, passes=16, fa=1 - 2 ** -12, fb=2 ** -12)
        r1 = ctx1.stressor("valu_f32", 1.0, ws=ws1, dst=out32[0], **o).stop()
        s1 = ctx1.stressor("valu_f32", 1.0, ws=ws1, dst=out32[0], **o)
        s2 = ctx2.stressor("valu_f32", 1.0, ws=ws2, dst=out32[1], **o)
        a, b = s1.stop(), s2.stop()
        row = {"ilp": ilp, "alone_ms": round(r1.window_ns / 1e6, 4),
               "colocated_ms_each": round((a.window_ns + b.window_ns) / 2 / 1e6, 4),
               "slowdown_each": round((a.window_ns + b.window_ns) / 2 / r1.window_ns, 3),
               "alone_pct_peak": round(r1.pct_of_peak, 1)}
        out["fp32_fma"].append(row)
        log(json.dumps(row))
    ctx1.close()
    ctx2.close()
    _emit(out, args)


def run_ldsstride(args):
    """Shared-memory interference (Section 4.4.1, Figure 4 analog): GEMM
    victims (BF16, dims 1024 and 2048) against the LDS stressor with 32-bit
    accesses at stride 1..64 words (bank-conflict degree), same CUs."""
    import torch
    from paper_2501_16909_amd import coloc
    ctx = coloc.Context(0)
    dev = ctx.device
    ops = stressor_operands(dev)
    ws = torch.empty(WS_BYTES, dtype=torch.uint8, device=dev)
    out = {"metric": "GEMM slowdown vs LDS stressor bank-conflict stride",
           "config": {"workload": "BF16 GEMM n = 1024 and 2048 (own MFMA kernel); LDS stressor 64 KiB per WG, "
                                  "256 threads, one WG per CU, 32-bit accesses at stride s words"}, "rows": []}
    victims = {n: _gemm_victim(ctx, dev, n) for n in (1024, 2048)}
    for stride in (1, 2, 4, 8, 16, 32, 64):
        o = dict(ops["lds"], vec=1, knob=stride, threads=256, wg_per_cu=1)
        rep = ctx.stressor("lds", 1.0, ws=ws, passes=2, **o).stop()
        row = {"stride": stride, "lds_tbs_alone": round(rep.units / rep.kernel_ns / 1e3, 2)}
        for n, d in victims.items():
            row[f"gemm_{n}"] = _cell(ctx.measure_sensitivity(d, ["lds"], [o], [1.0], reps=args.reps, warmups=2,
                                                             ws=ws, deadline_ms=args.deadline_ms)[0])
        out["rows"].append(row)
        log(json.dumps(row))
    ctx.close()
    _emit(out, args)


LLAMA31_8B = dict(hidden=4096, n_q=32, n_kv=8, head_dim=128, ffn=14336, vocab=128256, layers=32,
                 eps=1e-5, rope_base=500000.0)


def run_decode(args):
    """Synthetic decode step as the victim (the LLM decode victims of
    Sections 4.2-4.4 with random weights; per-kernel breakdown as in
    Fig. 5): Llama-3.1-8B shapes, BF16 weights and KV cache, 4096-entry
    cache per sequence.  Alone: step p50/p90 (replayed as a HIP graph, and
    as plain launches), HBM bytes per step and the achieved rate, per-kernel
    medians (launches with their own events).  Then the step beside each
    stressor (shared CUs, CU fraction 0.25 / 0.5 / 1.0; duty 25 / 50 % on
    every CU): p50/p90 step slowdown (graph) and the kernels that lose most
    (per-kernel events)."""
    import torch
    import synth
    from paper_2501_16909_amd import coloc
    ctx = coloc.Context(0)
    dev = ctx.device
    batch = args.batch
    cfg = dict(LLAMA31_8B, batch=batch, max_ctx=4096)
    pos = [4095 - 1024 * (b % 4) for b in range(batch)]     # ragged contexts
    model = coloc.DecodeModel(ctx, cfg, pos, synth.seed_for(5, 0))
    lay = model.layout
    nsteps = max(args.steps, 20)

    def steps_in(flags):
        model.set_flags(flags)
        for _ in range(args.warmup + 3):
            ctx.decode_step(model)
        return [ctx.decode_step(model) for _ in range(nsteps)]

    graph = np.array([r["step_ns"] for r in steps_in(coloc.DECODE_GRAPH)])
    plain = np.array([r["step_ns"] for r in steps_in(0)])
    timed = steps_in(coloc.DECODE_KERNEL_TIMES)
    kern = {k: float(np.median([r["kernel_ns"][k] for r in timed])) for k in coloc.DECODE_KERNELS}
    kv_read = sum((p + 1) for p in pos) * cfg["n_kv"] * cfg["head_dim"] * 2 * 2 * cfg["layers"]
    weight_bytes = 2 * int(lay.weight_elems)
    step_bytes = weight_bytes + kv_read
    p50 = float(np.median(graph))
    gemv_ns = sum(kern[k] for k in ("qkv", "oproj", "gate_up", "down", "lm_head"))
    alone = {"step_us_p50": round(p50 / 1e3, 1), "step_us_p90": round(float(np.quantile(graph, 0.9)) / 1e3, 1),
             "step_us_p50_plain_launches": round(float(np.median(plain)) / 1e3, 1),
             "step_us_p50_timed_launches": round(float(np.median([r["step_ns"] for r in timed])) / 1e3, 1),
             "hbm_bytes_per_step": step_bytes, "achieved_gb_s": round(step_bytes / p50, 1),
             "pct_of_hbm_peak": round(100 * step_bytes / p50 / 8000.0, 1),
             "gemv_gb_s": round(weight_bytes / gemv_ns, 1),
             "kernel_us": {k: round(v / 1e3, 1) for k, v in kern.items()}}
    log("decode alone: " + json.dumps(alone))
    ops = stressor_operands(dev)
    ws = torch.empty(WS_BYTES, dtype=torch.uint8, device=dev)
    res = ["hbm", "l2", "mall", "lds", "valu_f32", "mfma_bf16", "ptrchase"]
    rows = []
    for axis, levels in (("cu", [0.25, 0.5, 1.0]), ("duty", [25, 50])):
        for lv in levels:
            xs = [lv] if axis == "cu" else [1.0]
            opts = [dict(ops[r], duty=(lv if axis == "duty" else 100)) for r in res]
            model.set_flags(coloc.DECODE_GRAPH)
            steps = ctx.measure_decode(model, res, opts, xs, reps=args.reps, warmups=2, ws=ws,
                                       deadline_ms=max(args.deadline_ms, 500))
            model.set_flags(coloc.DECODE_KERNEL_TIMES)
            kcells = ctx.measure_decode(model, res, opts, xs, reps=max(3, args.reps // 2), warmups=1, ws=ws,
                                        deadline_ms=max(args.deadline_ms, 500))
            for c, kcell in zip(steps, kcells):
                ka, kc = kcell["kernel_alone_ns"], kcell["kernel_col_ns"]
                worst = sorted(((kc[k] / ka[k], k) for k in ka if ka[k] > 0), reverse=True)[:3]
                rows.append({"resource": c["resource"], "axis": axis, "level": lv,
                             "slowdown_p50": round(c["step_col_p50"] / c["step_alone_p50"], 3),
                             "slowdown_p90": round(c["step_col_p90"] / c["step_alone_p90"], 3),
                             "stressor_pct_peak": round(c["stressor_pct_peak"], 1),
                             "worst_kernels": [[k, round(v, 2)] for v, k in worst],
                             "window_covered": bool(c["window_covered"] and kcell["window_covered"]),
                             "output_equal": bool(c["output_equal"] and kcell["output_equal"])})
                log(json.dumps(rows[-1]))
    out = {"metric": "decode-step victim: step time alone and p50/p90 slowdown per stressor",
           "config": {"workload": f"synthetic decode step, Llama-3.1-8B shapes (32 layers, 4096 hidden, 32/8 "
                                  f"heads x 128, FFN 14336, vocab 128256), BF16 weights, batch {batch}, "
                                  f"cache positions {pos}", "model": "Llama-3.1-8B shapes, random weights"},
           "alone": alone, "cells": rows, "queue_pair_check": ctx.queue_stats()}
    ctx.close()
    _emit(out, args)


def _emit(out, args):
    print(json.dumps(out), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(out, f)



def run_queues(args):
    """Hardware-queue interference: a victim beside an idle kernel (the
    occupancy hog sleeping on the stressor's CUs, 1 KiB of LDS per
    work-group) in several launch shapes, with and without the queue-pair
    check, over fresh contexts whose CU-masked queues are created in seeded
    random orders.  Without the check the slowdown measures the queues
    alone; with it, what remains after the harness picks its queues."""
    import torch
    import synth
    from paper_2501_16909_amd import coloc
    dev = torch.device("cuda:0")
    n = 8192
    w = torch.from_numpy(synth.normal_f32(synth.seed_for(2, synth.BUF_GEMV_W), n * n, sigma=0.02)).to(dev)
    x = torch.from_numpy(synth.normal_f32(synth.seed_for(2, synth.BUF_GEMV_X), n)).to(dev)
    shapes = [(64, 1), (256, 1), (256, 4), (1024, 1)]
    rng = np.random.default_rng(16909)
    runs = []
    t0 = time.perf_counter()
    for c in range(args.contexts):
        ctx = coloc.Context(0)
        qw, _ = ctx.quantize(w, "bf16")
        qx, _ = ctx.quantize(x, "bf16")
        w3 = qw.repeat(3)
        y = torch.empty(n, dtype=torch.float32, device=dev)
        d = ctx.gemv_desc(w3, qx, y, n, n, copies=3)
        masks = [(xx, comp) for xx in (0.25, 0.5, 0.75) for comp in (False, True)] + [(1.0, False)]
        order = [masks[i] for i in rng.permutation(len(masks))]
        for xx, comp in order:
            ctx.probe_placement(ctx.cu_mask(xx, comp)[0], 64)
        run = {"context": c, "queue_order": [f"{'complement ' if comp else ''}{xx:g}" for xx, comp in order],
               "raw": {}, "checked": {}}
        for placement in ("disjoint", "shared"):
            for th, wg in shapes:
                o = dict(threads=th, wg_per_cu=wg, knob=1)
                cell = ctx.measure_sensitivity(d, ["occupancy"], [o], [0.5], reps=args.reps, warmups=3,
                                               placement=placement, queue_check=False)[0]
                run["raw"][f"{placement} {th}x{wg}"] = round(cell["slowdown"], 3)
            cell = ctx.measure_sensitivity(d, ["occupancy"], [dict(threads=256, wg_per_cu=1, knob=1)], [0.5],
                                           reps=args.reps, warmups=3, placement=placement)[0]
            run["checked"][f"{placement} 256x1"] = round(cell["slowdown"], 3)
        run["queue_pair_check"] = ctx.queue_stats()
        log(json.dumps(run))
        runs.append(run)
        del w3, qw, qx, y
        ctx.close()
    summary = {}
    for key in runs[0]["raw"]:
        v = [r["raw"][key] for r in runs]
        summary["raw " + key] = {"min": min(v), "median": float(np.median(v)), "max": max(v)}
    for key in runs[0]["checked"]:
        v = [r["checked"][key] for r in runs]
        summary["checked " + key] = {"min": min(v), "median": float(np.median(v)), "max": max(v)}
    out = {"metric": "victim slowdown beside an idle kernel on another hardware queue",
           "config": {"workload": "BF16 GEMV 8192^2 (3 rotating copies) victim; sleeping occupancy hog on the "
                                  "other half of the CUs (disjoint) or on half the CUs (shared); intensity 0.5",
                      "contexts": args.contexts, "reps": args.reps},
           "runs": runs, "summary": summary, "seconds": round(time.perf_counter() - t0, 1)}
    _emit(out, args)


def median_profiles(runs):
    """Point-wise median of several profile measurements (curves and
    pressures); the other fields come from the first run."""
    out = {}
    for kind, first in runs[0].items():
        p = dict(first)
        p["sens"] = {r: [float(np.median([run[kind]["sens"][r][i] for run in runs])) for i in range(len(curve))]
                     for r, curve in first["sens"].items()}
        p["press"] = {r: float(np.median([run[kind]["press"][r] for run in runs])) for r in first["press"]}
        out[kind] = p
    return out


def library_profiles(profiles, reads):
    """Profiles in the library's form (ci_profile_t through coloc.make_profiles):
    each kind's curves and pressures plus its curve and pressure against the
    read-only HBM mix, for read/write-aware pricing."""
    out = {}
    for kind, p in profiles.items():
        q = dict(p)
        q["sens_hbm_read"] = reads[kind]["sens"]["hbm"]
        q["press_hbm_read"] = reads[kind]["press"]["hbm"]
        out[kind] = q
    return out


def predicted_pair_slowdown(profiles, a, b, read_profiles=None, mall_profiles=None):
    """Product over resources of max(1, curve_A(pressure of B)).  With
    read_profiles (HBM curves and pressures against the read-only mix), a
    co-runner whose HBM traffic is mostly reads (write fraction below 1/6)
    is priced on the read-only curve instead of the triad's.  With
    mall_profiles, a co-runner whose working set fits the Infinity Cache is
    priced on the curve against the Infinity-Cache stressor instead."""
    out = 1.0
    pts = np.array(INTENSITIES)
    for r, curve in profiles[a]["sens"].items():
        x = profiles[b]["press"].get(r, 0.0)
        if r == "hbm" and mall_profiles is not None and KIND_FOOTPRINT[b] <= MALL_BYTES:
            curve, x = mall_profiles[a]["sens"]["mall"], mall_profiles[b]["press"]["mall"]
        elif r == "hbm" and read_profiles is not None and profiles[b]["hbm_write_frac"] < 1 / 6:
            curve, x = read_profiles[a]["sens"]["hbm"], read_profiles[b]["press"]["hbm"]
        x = min(1.0, max(0.0, x))
        out *= max(1.0, float(np.interp(x, pts, curve)))
    return out


def estimator_victim(ctx, kind: str, seed: int):
    """One instance of a request kind at the estimator's sizes: BF16 GEMM
    2048^3, BF16 GEMV 8192^2, FP32 triad 2^24 (uniform inputs from `seed`)."""
    import torch
    import synth
    dev = ctx.device
    if kind == "gemm":
        g = 2048
        A = torch.from_numpy(synth.uniform_f32(seed, g * g)).to(dev)
        B = torch.from_numpy(synth.uniform_f32(seed + 1, g * g)).to(dev)
        qa, _ = ctx.quantize(A, "bf16")
        qb, _ = ctx.quantize(B, "bf16")
        return ctx.gemm_desc(qa, qb, torch.empty((g, g), dtype=torch.float32, device=dev), "bf16", g, g, g)
    if kind == "gemv":
        n = 8192
        W = torch.from_numpy(synth.uniform_f32(seed, n * n)).to(dev)
        X = torch.from_numpy(synth.uniform_f32(seed + 1, n)).to(dev)
        qw, _ = ctx.quantize(W, "bf16")
        qx, _ = ctx.quantize(X, "bf16")
        return ctx.gemv_desc(qw, qx, torch.empty(n, dtype=torch.float32, device=dev), n, n)
    t = 1 << 24
    tb = torch.from_numpy(synth.uniform_f32(seed, t)).to(dev)
    tc = torch.from_numpy(synth.uniform_f32(seed + 1, t)).to(dev)
    return ctx.triad_desc(tb, tc, torch.empty_like(tb), passes=1)


def measure_pair(ctx, da, db, reps: int, streams: int = 3, max_attempts: int = 8):
    """Slowdown of victim A while B runs beside it.  B goes on a fresh
    stream, bracketed by two device stamps; a colocated run counts only if
    B's stamps cover A's whole window (A started after B's first launches,
    ended before B's last one).  Two kernels on two queues can also slow
    each other through the queues alone, which only adds: the pair is
    measured on up to `streams` streams that gave covered runs and the
    lowest ratio is kept.  Returns (lowest, per-stream ratios, streams tried)."""
    import torch
    dev = ctx.device
    stamps = torch.zeros(2, dtype=torch.int64, device=dev)
    started = torch.cuda.Event()
    t_a = float(np.median([ctx.victim_run(da).time_ns for _ in range(5)]))
    tb_alone = float(np.median([ctx.victim_run(db).time_ns for _ in range(3)]))
    count = int(min(4000, max(20, 6.0 * t_a / tb_alone)))
    trials, attempts = [], 0
    while len(trials) < streams and attempts < max_attempts:
        attempts += 1
        side = torch.cuda.Stream(device=dev)
        alone, col = [], []
        for r in range(reps):
            if r % 2 == 0:
                alone.append(ctx.victim_run(da).time_ns)
            side.synchronize()
            # a short first batch, then the timed victim starts while the
            # main batch runs
            ctx.victim_enqueue(db, side, 2)
            ctx.stamp(stamps[0:1], side)
            started.record(side)
            ctx.victim_enqueue(db, side, count)
            ctx.stamp(stamps[1:2], side)
            while not started.query():
                pass
            out_a = ctx.victim_run(da)
            side.synchronize()
            s0, s1 = (int(v) for v in stamps.cpu().tolist())
            if s0 <= out_a.t_begin and s1 >= out_a.t_end:
                col.append(out_a.time_ns)
            if r % 2 == 1:
                alone.append(ctx.victim_run(da).time_ns)
        if len(col) * 2 > reps:
            trials.append(float(np.median(col) / np.median(alone)))
    if not trials:
        raise RuntimeError("estimator pair: the co-runner never covered the victim")
    return min(trials), trials, attempts


def run_estimator(args):
    """Kernel-level interference estimator (Section 5.1), validated on
    workload pairs: predict the slowdown of victim A while victim B runs
    beside it (B enqueued back to back on a second stream for longer than A
    runs), from A's sensitivity curves and B's standalone pressure, and
    compare with the measured slowdown (medians of counterbalanced runs,
    lowest of three co-runner streams)."""
    from paper_2501_16909_amd import coloc
    ctx = coloc.Context(0)
    def profiles(**kw):
        # the point-wise median over --profile-runs independent measurements
        runs = [serve_profiles(ctx, args, **kw) for _ in range(max(1, args.profile_runs))]
        return median_profiles(runs)
    axes = {"cu": profiles(axis="cu"), "duty": profiles(axis="duty")}
    # HBM curves against the read-only mix, for read-mostly co-runners
    read_axes = {ax: profiles(axis=ax, hbm_mix="read", res=("hbm",)) for ax in axes}
    # curves against the Infinity-Cache stressor, for co-runners that fit it
    mall_axes = {ax: profiles(axis=ax, res=("mall",)) for ax in axes}
    log("profiles: " + json.dumps(axes))
    log("read-mix HBM profiles: " + json.dumps(read_axes))
    log("Infinity-Cache profiles: " + json.dumps(mall_axes))
    lib_profiles = library_profiles(axes["duty"], read_axes["duty"])
    kinds = ["gemm", "gemv", "triad"]
    # two independent instances of each kind (A's buffers and B's buffers)
    A = {k: estimator_victim(ctx, k, 7000 + 10 * i) for i, k in enumerate(kinds)}
    B = {k: estimator_victim(ctx, k, 8000 + 10 * i) for i, k in enumerate(kinds)}
    rows = []
    for a in kinds:
        for b in kinds:
            meas, trials, attempts = measure_pair(ctx, A[a], B[b], args.reps)
            row = {"victim": a, "corunner": b, "measured": round(meas, 3),
                   "measured_trials": [round(t, 3) for t in trials], "stream_attempts": attempts}
            for ax, prof in axes.items():
                for name, rp, mp in ((ax, None, None), (ax + "_mix", read_axes[ax], None),
                                     (ax + "_fit", read_axes[ax], mall_axes[ax])):
                    pred = predicted_pair_slowdown(prof, a, b, rp, mp)
                    row[f"predicted_{name}"] = round(pred, 3)
                    row[f"rel_err_{name}"] = round(abs(pred - meas) / meas, 3)
            # the library's estimator (ci_predict_slowdown, what admission
            # uses) on the duty-axis profiles with read/write-aware pricing
            pred = coloc.predict_slowdown(lib_profiles, a, [b])
            row["predicted_library"] = round(pred, 3)
            row["rel_err_library"] = round(abs(pred - meas) / meas, 3)
            rows.append(row)
            log(json.dumps(row))
    rank = lambda v: np.argsort(np.argsort(v))
    m = np.array([r["measured"] for r in rows])
    summary = {}
    for ax in [a for x in axes for a in (x, x + "_mix", x + "_fit")] + ["library"]:
        err = np.array([r[f"rel_err_{ax}"] for r in rows])
        p = np.array([r[f"predicted_{ax}"] for r in rows])
        summary[ax] = {"mean_rel_err": round(float(err.mean()), 3), "max_rel_err": round(float(err.max()), 3),
                       "spearman": float(np.corrcoef(rank(m), rank(p))[0, 1]) if len(rows) > 2 else None}
    out = {"metric": "estimator error on workload pairs",
           "config": {"workload": "victims BF16 GEMM 2048^3, BF16 GEMV 8192^2, FP32 triad 2^24; co-runner "
                                  "enqueued back to back on a second stream; shared CUs",
                      "model": "product over HBM / BF16-MFMA / LDS of max(1, sensitivity curve at the "
                               "co-runner's standalone pressure); curves on two intensity axes: CU "
                               "fraction at full rate ('cu') and duty cycle on every CU ('duty'); "
                               "'_mix': read-mostly co-runners priced on the read-only HBM curve; "
                               "'_fit': also, co-runners whose working set fits the 256 MB Infinity "
                               "Cache priced on the Infinity-Cache stressor's curve; 'library': "
                               "ci_predict_slowdown on the duty-axis profiles (read/write-aware)"},
           "profile_runs": max(1, args.profile_runs),
           "pairs": rows, "axes": summary, "profiles": axes, "read_mix_profiles": read_axes,
           "mall_profiles": mall_axes}
    ctx.close()
    _emit(out, args)


def run_suite_counters(args):
    """Each stressor of the suite once, fixed work, no colocation: the run
    the per-stressor hardware-counter passes profile."""
    import torch
    from paper_2501_16909_amd import coloc
    dev = torch.device("cuda:0")
    ctx = coloc.Context(0)
    suite = Suite(ctx, dev)
    for name, opts, unit, scale in suite.items:
        rep = ctx.stressor(suite_resource(name), 1.0, ws=suite.ws, **opts).stop()
        log(f"{name}: {rep.units / (rep.kernel_ns * 1e-9) / scale:.2f} {unit}")
    ctx.close()
    print(json.dumps({"counters_run": "stressor suite, one fixed-work launch each"}), flush=True)


def run_gemm_counters(args):
    """Short run for hardware-counter passes on the GEMM victim: BF16
    M = N = K = 4096 (the sweep's GEMM shape, uniform inputs), three launches."""
    import torch
    import synth
    from paper_2501_16909_amd import coloc
    dev = torch.device("cuda:0")
    ctx = coloc.Context(0)
    g = 4096
    a = torch.empty(g * g, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    synth.device_fill_uniform_f32(a.data_ptr(), g * g, synth.seed_for(2, synth.BUF_GEMM_A))
    synth.device_fill_uniform_f32(b.data_ptr(), g * g, synth.seed_for(2, synth.BUF_GEMM_B))
    torch.cuda.synchronize()
    qa, sa = ctx.quantize(a, "bf16")
    qb, sb = ctx.quantize(b, "bf16")
    c = torch.empty((g, g), dtype=torch.float32, device=dev)
    d = ctx.gemm_desc(qa.view(g, g), qb.view(g, g), c, "bf16", g, g, g, sa, sb)
    for _ in range(3):
        r = ctx.victim_run(d)
        log(f"gemm bf16 4096^3: {2.0 * g ** 3 / r.time_ns / 1e3:.1f} TF")
    ctx.close()
    print(json.dumps({"counters_run": "gemm bf16 4096^3 x3"}), flush=True)


def run_chase_latency(args):
    """Pointer-chase latency with few chains in flight: one 64-lane wave on
    one CU of each XCD (512 chains, one per lane), each following a uniformly
    random single cycle (Sattolo-equivalent table, seeded) for 8192 hops;
    ns per hop = the launch's window over the hops one chain makes.  Tables
    of 2^20, 2^24 and 2^27 entries (4 MiB: L2-sized; 64 MiB: inside the
    Infinity Cache; 512 MiB: beyond it, from HBM).  The end indices are
    checked against a host walk of the same table for 8 chains."""
    import torch
    import synth
    from paper_2501_16909_amd import coloc
    dev = torch.device("cuda:0")
    ctx = coloc.Context(0)
    ws = torch.empty(WS_BYTES, dtype=torch.uint8, device=dev)
    hops = 8192
    rows = []
    for lg in (20, 24, 27):
        n = 1 << lg
        nxt = synth.random_cycle_u32(synth.seed_for(6, synth.BUF_CHASE) + lg, n)
        t_next = torch.from_numpy(nxt.view(np.int32)).to(dev)
        end = torch.empty(8 * 64, dtype=torch.int32, device=dev)
        o = dict(src0=t_next, n=n, dst=end, threads=64, wg_per_cu=1, knob=1, iters=hops, passes=1)
        ctx.stressor("ptrchase", 1 / 32, ws=ws, **o).stop()           # untimed: fills the caches and TLBs
        rep = ctx.stressor("ptrchase", 1 / 32, ws=ws, **o).stop()
        got = end.cpu().numpy().view(np.uint32)
        chains = rep.grid * 64
        ok = True
        for c in range(0, chains, chains // 8):                       # host walk of 8 chains
            i = np.uint32(c * (n // chains))
            for _ in range(hops):
                i = nxt[i]
            ok &= bool(got[c] == i)
        row = {"entries": n, "mib": n * 4 >> 20, "chains": chains, "hops_per_chain": hops,
               "ns_per_hop": round(rep.window_ns / hops, 1), "ghops_per_s": round(rep.units / rep.window_ns, 2),
               "end_indices_match_host_walk": ok}
        rows.append(row)
        log(json.dumps(row))
        del t_next
        torch.cuda.empty_cache()
    ctx.close()
    _emit({"metric": "pointer-chase latency, one wave per XCD", "rows": rows}, args)


def run_hbm_references(args):
    """Short run for a kernel trace: the HBM stressor's four traffic mixes
    over N = 2^30 FP32 (fixed work, one pass per launch) and, over the same
    arrays as independent references, the framework's own elementwise
    triad (torch.add(b, c, alpha=3)), tensor copy and fill, six launches
    each.  `--config reference-summary` turns the trace into
    profiles/hbm_references_n2e30_kernel_trace.md."""
    import torch
    import synth
    from paper_2501_16909_amd import coloc
    dev = torch.device("cuda:0")
    ctx = coloc.Context(0)
    n = 1 << 30
    hb = torch.empty(n, dtype=torch.float32, device=dev)
    hc, ha = torch.empty_like(hb), torch.empty_like(hb)
    synth.device_fill_uniform_f32(hb.data_ptr(), n, synth.seed_for(1, synth.BUF_B))
    synth.device_fill_uniform_f32(hc.data_ptr(), n, synth.seed_for(1, synth.BUF_C))
    torch.cuda.synchronize()
    ws = torch.empty(WS_BYTES, dtype=torch.uint8, device=dev)
    mixes = [("triad", dict(src0=hb, src1=hc, dst=ha)), ("read", dict(src0=hb, src1=hc)),
             ("copy", dict(src0=hb, dst=ha)), ("write", dict(dst=ha))]
    for mix, ops in mixes:
        for _ in range(6):
            rep = ctx.stressor("hbm", 1.0, ws=ws, n=n, passes=1, knob=coloc.HBM_MIX[mix], **ops).stop()
        log(f"hbm {mix}: {rep.achieved / 1e9:.0f} GB/s")
    ctx.close()
    # each pass over the arrays as two launches of 2^29 elements: the
    # framework splits a launch whose offsets pass 2^31 bytes anyway, and
    # this way every traced launch covers a known half
    h = n // 2
    for name, fn in (("torch.add triad", lambda lo, hi: torch.add(hb[lo:hi], hc[lo:hi], alpha=3.0, out=ha[lo:hi])),
                     ("copy_", lambda lo, hi: ha[lo:hi].copy_(hb[lo:hi])),
                     ("fill_", lambda lo, hi: ha[lo:hi].fill_(1.0))):
        for _ in range(6):
            fn(0, h)
            fn(h, n)
        torch.cuda.synchronize()
        log(f"{name} done")
    print(json.dumps({"references_run": "hbm mixes and framework kernels over 2^30 FP32, 6 launches each"}),
          flush=True)


# ---------------------------------------------------------------- profiles
# Summaries of rocprofv3 databases (rocpd SQLite) into the text files kept
# under profiles/.  They run on any host: no GPU, no library.

TCC_CHANNELS = 128      # 16 L2 channels per XCD x 8 XCDs; per-channel counters are summed over them
GRBM_INSTANCES = 8      # GRBM_GUI_ACTIVE is summed over the 8 XCDs

# the fixed-work launches of `--config counters`, by kernel
HBM_COUNTER_KERNELS = [("triad", "stream_stressor<1u, true, 4, true>", 12),
                       ("read", "strided_stressor<2u, true, 4>", 8),
                       ("copy", "stream_stressor<3u, true, 4, true>", 8),
                       ("write", "stream_stressor<4u, true, 4, true>", 4)]


def _short_kernel(name: str) -> str:
    n = name.replace("void ", "").replace("ci::(anonymous namespace)::", "").replace("(anonymous namespace)::", "")
    depth = 0
    for i, ch in enumerate(n):      # cut the argument list (the first "(" outside template brackets)
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return n[:i]
    return n


def _pmc_dispatches(db):
    """[{name, grid, wg, start, end, ctr: {counter: value}}] in dispatch order."""
    import sqlite3
    con = sqlite3.connect(db)
    rows = con.execute("select dispatch_id, kernel_name, grid_size, workgroup_size, counter_name, sum(value), "
                       "min(start), max(end) from counters_collection group by dispatch_id, counter_name "
                       "order by dispatch_id").fetchall()
    con.close()
    out = {}
    for did, name, grid, wg, ctr, val, t0, t1 in rows:
        d = out.setdefault(did, {"name": _short_kernel(name), "grid": int(grid), "wg": int(wg), "start": t0,
                                 "end": t1, "ctr": {}})
        d["ctr"][ctr] = float(val)
    return [out[k] for k in sorted(out)]


def run_counter_summary(args):
    """HBM traffic and DRAM-side counters of `--config counters` from the
    rocprofv3 --pmc databases given with --dbs (one counter set per run):
    writes profiles/hbm_triad_n2e30_counters.{json,md}."""
    n = 1 << 30
    per = {mix: [] for mix, _, _ in HBM_COUNTER_KERNELS}
    calib = []
    for db in args.dbs:
        seen = {mix: 0 for mix in per}
        ncal = 0
        copies = [d for d in _pmc_dispatches(db) if d["name"] == "__amd_rocclr_copyBuffer"]
        big = max((d["grid"] for d in copies), default=0)
        for d in _pmc_dispatches(db):
            for mix, kname, _ in HBM_COUNTER_KERNELS:
                if d["name"] == kname and d["grid"] == 256 * 512:
                    if seen[mix] == len(per[mix]):
                        per[mix].append({})
                    per[mix][seen[mix]].update(d["ctr"])
                    seen[mix] += 1
            if d["name"] == "__amd_rocclr_copyBuffer" and d["grid"] == big and big > 0:
                if ncal == len(calib):
                    calib.append({})
                calib[ncal].update(d["ctr"])
                ncal += 1
    mean = lambda xs: float(np.mean(xs)) if xs else None
    gib = float(1 << 30)
    ff = gib / (1024.0 * mean([c["FETCH_SIZE"] for c in calib if "FETCH_SIZE" in c]))
    wf = gib / (1024.0 * mean([c["WRITE_SIZE"] for c in calib if "WRITE_SIZE" in c]))
    mixes = {}
    for mix, kname, bpe in HBM_COUNTER_KERNELS:
        ls = per[mix]
        get = lambda k: mean([l[k] for l in ls if k in l])
        fetch, write = get("FETCH_SIZE"), get("WRITE_SIZE")
        cyc = get("GRBM_GUI_ACTIVE") / GRBM_INSTANCES if get("GRBM_GUI_ACTIVE") else None
        m = {"kernel": kname, "launches": len(ls), "fetch_kib": fetch, "write_kib": write,
             "traffic_bytes": round(fetch * 1024 * ff + write * 1024 * wf),
             "algorithmic_bytes": bpe * n,
             "rdreq": get("TCC_EA0_RDREQ"), "rdreq_128b": get("TCC_EA0_RDREQ_128B"),
             "rdreq_64b": get("TCC_EA0_RDREQ_64B"), "rdreq_32b": get("TCC_EA0_RDREQ_32B"),
             "wrreq": get("TCC_EA0_WRREQ"), "wrreq_64b": get("TCC_EA0_WRREQ_64B"),
             "cycles_per_xcd": cyc}
        if cyc:
            ch = TCC_CHANNELS * cyc
            m["tcc_busy_frac"] = get("TCC_BUSY") / ch
            m["rd_credit_stall_frac"] = get("TCC_EA0_RDREQ_DRAM_CREDIT_STALL") / ch
            m["wr_credit_stall_frac"] = get("TCC_EA0_WRREQ_DRAM_CREDIT_STALL") / ch
            m["reads_in_flight"] = get("TCC_EA0_RDREQ_LEVEL") / cyc
            m["writes_in_flight"] = get("TCC_EA0_WRREQ_LEVEL") / cyc
            if m["rdreq"] and m["rdreq"] > 1e6:
                m["read_latency_cycles"] = get("TCC_EA0_RDREQ_LEVEL") / m["rdreq"]
            if m["wrreq"] and m["wrreq"] > 1e6:
                m["write_latency_cycles"] = get("TCC_EA0_WRREQ_LEVEL") / m["wrreq"]
        mixes[mix] = m
    t = mixes["triad"]
    out = {"kernel": "stream_stressor<1u, true, 4, true> (HBM stressor, triad mix, N=2^30 FP32, one pass, "
                     "256 work-groups x 512 threads)",
           "kernel_sources": HBM_KERNEL_SOURCES,
           "kernel_source_sha": sha_of(*[os.path.join(ROOT, p) for p in HBM_KERNEL_SOURCES]),
           "commands": args.cmd,
           "calibration_copy_1GiB": {"fetch_factor": round(ff, 4), "write_factor": round(wf, 4),
                                     "note": "the runtime's 1 GiB device-to-device copy (1 GiB read, 1 GiB "
                                             "written): the factors scale each counter to bytes"},
           "traffic_bytes_per_launch": t["traffic_bytes"],
           "algorithmic_bytes_per_launch": t["algorithmic_bytes"],
           "traffic_over_algorithmic": round(t["traffic_bytes"] / t["algorithmic_bytes"], 4),
           "mixes": mixes}
    base = os.path.join(ROOT, "profiles", "hbm_triad_n2e30_counters")
    with open(base + ".json", "w") as f:
        json.dump(out, f, indent=1)
    L = ["# HBM traffic and DRAM-side counters of the HBM stressor (N = 2^30 FP32, one pass per launch)", "",
         "Commands (repository root, one MI355X; one counter set per run), then the summary:", "", "```"]
    L += args.cmd + [" ".join(["python3 bench.py --config counter-summary --dbs"] + list(args.dbs)), "```", "",
                     "`bench.py --config counters` launches the HBM stressor's triad mix over N = 2^30 twice "
                     "(256 work-groups x 512 threads, one pass each), its read-only, copy and write-only "
                     "mixes once each, then the runtime's 1 GiB device-to-device copy twice (the "
                     "calibration kernel).", "",
                     f"Calibration: FETCH_SIZE x {ff:.4f} and WRITE_SIZE x {wf:.4f} give bytes.", "",
                     "| mix | kernel | traffic GiB (algorithmic) | 128 B reads | 64 B writes | L2 channels busy | "
                     "DRAM credit stall rd / wr | reads in flight | read latency (cycles) |",
                     "|---|---|---|---|---|---|---|---|---|"]
    for mix, m in mixes.items():
        L.append(f"| {mix} | `{m['kernel']}` | {m['traffic_bytes'] / gib:.3f} ({m['algorithmic_bytes'] / gib:.0f}) | "
                 f"{(m['rdreq_128b'] or 0) / 1e6:.2f} M | {(m['wrreq_64b'] or 0) / 1e6:.2f} M | "
                 f"{100 * m.get('tcc_busy_frac', float('nan')):.1f} % | "
                 f"{100 * m.get('rd_credit_stall_frac', float('nan')):.1f} / "
                 f"{100 * m.get('wr_credit_stall_frac', float('nan')):.1f} % | "
                 f"{m.get('reads_in_flight', float('nan')):.0f} | {m.get('read_latency_cycles', float('nan')):.0f} |")
    L += ["", f"Triad traffic per launch {t['traffic_bytes']} bytes against {t['algorithmic_bytes']} algorithmic "
              f"(ratio {out['traffic_over_algorithmic']:.4f}): no re-reads, and no read of the output before "
              "it is written.", "",
          "Per-channel fractions divide by 128 L2 channels x GRBM_GUI_ACTIVE / 8 (the 8 XCDs' cycles); "
          "in-flight counts divide the accumulated TCC_EA0_*REQ_LEVEL by the same cycles; latency is "
          "in-flight / issue rate (Little's law).", "",
          "The summary holds for the kernel sources whose hash it records; the benchmark reports the "
          "traffic only while that hash matches."]
    with open(base + ".md", "w") as f:
        f.write("\n".join(L) + "\n")
    print(json.dumps({"written": [base + ".json", base + ".md"], "triad_traffic": t["traffic_bytes"]}))


def run_trace_summary(args):
    """Kernel-trace summary (per kernel and launch shape: calls, average,
    min, max, total) of one rocprofv3 --kernel-trace database, written to
    --md; --top keeps the rows with the largest totals; with --bench-json,
    the benchmark line's roofline kernel is checked against the trace's
    average launch time; with --window-ms, every launch longer than that
    (a stressor held through a run) is listed with the kernels that started
    and ended inside its window."""
    import sqlite3
    con = sqlite3.connect(args.dbs[0])
    rows = con.execute("select name, grid_x, workgroup_x, count(*), avg(duration), min(duration), max(duration), "
                       "sum(duration) from kernels group by name, grid_x, workgroup_x "
                       "order by sum(duration) desc").fetchall()
    windows = []
    if args.window_ms:
        for name, t0, t1, dur in con.execute("select name, start, end, duration from kernels where duration > ? "
                                             "order by start", (args.window_ms * 1e6,)).fetchall():
            inside = con.execute("select name, count(*) from kernels where start >= ? and end <= ? and "
                                 "not (start = ? and end = ?) group by name order by count(*) desc",
                                 (t0, t1, t0, t1)).fetchall()
            windows.append((name, dur, inside))
    con.close()
    total_kernels = len(rows)
    if args.top:
        rows = rows[:args.top]
    L = [f"# {args.title}", "", "Command (repository root, one MI355X), then the summary:", "", "```"]
    flags = (f" --top {args.top}" if args.top else "") + (f" --window-ms {args.window_ms:g}" if args.window_ms else "")
    L += args.cmd + [" ".join(["python3 bench.py --config trace-summary --dbs"] + list(args.dbs)) + flags, "```", "",
                     "| kernel | work-groups x threads | calls | avg us | min us | max us | total ms |",
                     "|---|---|---|---|---|---|---|"]
    for name, gx, wx, calls, avg, mn, mx, tot in rows:
        L.append(f"| `{_short_kernel(name)}` | {gx // max(wx, 1)} x {wx} | {calls} | {avg / 1e3:.2f} | "
                 f"{mn / 1e3:.2f} | {mx / 1e3:.2f} | {tot / 1e6:.3f} |")
    if len(rows) < total_kernels:
        L += ["", f"({len(rows)} of {total_kernels} kernel and launch-shape rows, by total time.)"]
    for name, dur, inside in windows:
        L += ["", f"Launch of `{_short_kernel(name)}` lasting {dur / 1e6:.1f} ms; kernels that started and ended "
                  f"inside its window: {sum(c for _, c in inside)}"]
        L += [f"- `{_short_kernel(n)}`: {c}" for n, c in inside]
    if args.bench_json:
        with open(args.bench_json) as f:
            line = json.loads(f.read().strip().splitlines()[-1])
        rf = line["roofline"]
        kname = rf["kernel"].split(":")[0]
        hit = [r for r in rows if _short_kernel(r[0]) == kname and r[1] == 256 * 512]
        if hit:
            avg_us = hit[0][4] / 1e3
            live_us = 12.0 * (1 << 30) / (rf["achieved"] * 1e9) * 1e6
            L += ["", f"Roofline kernel `{kname}`: the benchmark line of this run reports {rf['achieved']} GB/s, "
                      f"that is {live_us:.1f} us per launch (12 x 2^30 bytes); the trace's average over "
                      f"{hit[0][3]} launches (warm-up included) is {avg_us:.1f} us "
                      f"({12.0 * (1 << 30) / (avg_us * 1e-6) / 1e9:.0f} GB/s), "
                      f"{100 * (avg_us / live_us - 1):+.1f} %."]
    with open(args.md, "w") as f:
        f.write("\n".join(L) + "\n")
    print(json.dumps({"written": args.md, "kernels": len(rows)}))


# the kernels of `--config hbm-references`: bytes moved per element and what
# each is (the framework's kernels are recognised by their names)
HBM_REFERENCE_KERNELS = [("stream_stressor<1u, true, 4, true>", 12, "HBM stressor, triad mix (the roofline kernel)"),
                         ("strided_stressor<2u, true, 4>", 8, "HBM stressor, read-only mix"),
                         ("stream_stressor<3u, true, 4, true>", 8, "HBM stressor, copy mix"),
                         ("stream_stressor<4u, true, 4, true>", 4, "HBM stressor, write-only mix")]


def _reference_kind(short: str):
    """(bytes per element, elements per launch as a fraction of 2^30, what)."""
    for kname, per, what in HBM_REFERENCE_KERNELS:
        if short == kname:
            return per, 1.0, what
    if "Functor_add" in short:
        return 12, 0.5, "framework elementwise triad, torch.add(b, c, alpha=3, out=a)"
    if "copyBuffer" in short:
        return 8, 0.5, "framework tensor copy, a.copy_(b) (the runtime's device copy)"
    if "FillFunctor" in short:
        return 4, 0.5, "framework fill, a.fill_(1.0)"
    return None


def run_reference_summary(args):
    """HBM rates of `--config hbm-references` from one rocprofv3
    --kernel-trace database (--dbs): per reference kernel the median launch
    duration and the rate of its algorithmic bytes (the stressor's launches
    cover the 2^30 elements, the framework's a half each).  Writes
    profiles/hbm_references_n2e30_kernel_trace.md."""
    import sqlite3
    n = 1 << 30
    con = sqlite3.connect(args.dbs[0])
    rows = con.execute("select name, grid_x, workgroup_x, duration from kernels order by start").fetchall()
    con.close()
    groups = {}
    for name, gx, wx, dur in rows:
        short = _short_kernel(name)
        kind = _reference_kind(short)
        if kind is None or (kind[1] < 1 and dur < 100e3):   # the runtime's small copies are not references
            continue
        g = groups.setdefault((short, gx // max(wx, 1), wx), {"kind": kind, "durs": []})
        g["durs"].append(dur)
    cmd = " ".join(args.cmd) if args.cmd else "(not given)"
    md = args.md or os.path.join(ROOT, "profiles", "hbm_references_n2e30_kernel_trace.md")
    L = ["# HBM streaming over N = 2^30 FP32: the stressor's mixes and independent references", "",
         "Command (repository root, one MI355X), then the summary:", "", "```", cmd,
         f"python3 bench.py --config reference-summary --dbs {args.dbs[0]}", "```", "",
         "The launches of `bench.py --config hbm-references` over the 2^30-element arrays, by kernel: the "
         "median traced duration and the rate of the kernel's algorithmic bytes (triad 12, read-only and copy "
         "8, write-only and fill 4 bytes per element) against the 8 TB/s HBM peak. The stressor's launches "
         "each cover all 2^30 elements; the framework's kernels run each pass as two launches of 2^29 "
         "elements (it splits launches whose offsets pass 2^31 bytes).", "",
         "| kernel | what | work-groups x threads | elements per launch | launches | median us | GB/s | "
         "% of 8 TB/s |",
         "|---|---|---|---|---|---|---|---|"]
    for (short, wgs, wx), g in sorted(groups.items(), key=lambda kv: -kv[1]["kind"][0] * kv[1]["kind"][1]):
        per, frac, what = g["kind"]
        med = float(np.median(g["durs"]))
        rate = per * n * frac / med     # bytes per ns = GB/s
        L.append(f"| `{short}` | {what} | {wgs} x {wx} | 2^{29 if frac < 1 else 30} | {len(g['durs'])} | "
                 f"{med / 1e3:.1f} | {rate:.0f} | {rate / 80.0:.1f} |")
    with open(md, "w") as f:
        f.write("\n".join(L) + "\n")
    print(json.dumps({"written": md, "kernels": len(groups)}))


def run_gemm_counter_summary(args):
    """Counters of `--config gemm-counters` (three BF16 4096^3 launches of
    the ring kernel) from one rocprofv3 --pmc database (--dbs): writes
    profiles/gemm_bf16_4096_counters.md."""
    ds = [d for d in _pmc_dispatches(args.dbs[0]) if d["name"].startswith("gemm256d_kernel<")]
    if not ds:
        raise SystemExit(f"{args.dbs[0]}: no gemm256d_kernel dispatch")
    # further databases (--dbs A B C): the stall-breakdown counters of the same
    # launches, matched by launch order
    extra = [[d for d in _pmc_dispatches(db) if d["name"].startswith("gemm256d_kernel<")] for db in args.dbs[1:]]
    cmd = "\n".join(c.strip() for c in args.cmd) if args.cmd else "(not given)"
    L = ["# Hardware counters of the GEMM victim (BF16, M = N = K = 4096, ring kernel)", "",
         "Commands (repository root, one MI355X; one counter group per run), then the summary:", "", "```", cmd,
         f"python3 bench.py --config gemm-counter-summary --dbs {' '.join(args.dbs)}", "```", "",
         f"`bench.py --config gemm-counters` launches the BF16 4096³ GEMM three times (`{ds[0]['name']}`, "
         f"{ds[0]['grid'] // ds[0]['wg']} work-groups of {ds[0]['wg']} threads). Derived: active time = "
         "GRBM_GUI_ACTIVE / 8 XCDs / 2.4 GHz; MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES over active cycles x 1024 "
         "SIMDs; LDS B/clk/CU = SQ_INSTS_LDS x 1 KiB (each a 64-lane `ds_read_b128`) over active cycles x 256 "
         "CUs (ring fills by `global_load_lds` come on top, about 15 B/clk/CU); waits as fractions of "
         "SQ_WAVE_CYCLES.", "",
         "| launch | duration us (profiled) | active us | MFMA busy | LDS read B/clk/CU | waiting | "
         "waiting on LDS | LDS bank conflicts | LDS instructions | waves |",
         "|---|---|---|---|---|---|---|---|---|---|"]
    for i, d in enumerate(ds):
        c = d["ctr"]
        active = c["GRBM_GUI_ACTIVE"] / GRBM_INSTANCES
        L.append(f"| {i + 1} | {(d['end'] - d['start']) / 1e3:.1f} | {active / 2.4e3:.1f} | "
                 f"{c['SQ_VALU_MFMA_BUSY_CYCLES'] / (active * 1024):.3f} | "
                 f"{c['SQ_INSTS_LDS'] * 1024 / (active * 256):.1f} | "
                 f"{c['SQ_WAIT_ANY'] / c['SQ_WAVE_CYCLES']:.3f} | {c['SQ_WAIT_INST_LDS'] / c['SQ_WAVE_CYCLES']:.3f} | "
                 f"{c['SQ_LDS_BANK_CONFLICT']:.0f} | {c['SQ_INSTS_LDS']:.0f} | {c['SQ_WAVES']:.0f} |")
    L += ["", "Profiling slows the launches; the fractions are what matter: the matrix cores' busy share, the "
              "LDS fragment-load rate against the 256 B/clk/CU of the load path (`lds_stride_counters.md`), "
              "and the share of wave cycles spent waiting (on anything, and on LDS)."]
    if extra and all(len(e) == len(ds) for e in extra):
        L += ["", "Where a wave's cycles go (further counter runs of the same command; the SQ wave-cycle counters "
                  "share one unit, so the three shares add up to the whole): issuing = SQ_ACTIVE_INST_ANY, "
                  "waiting on a dependency or the barrier = SQ_WAIT_ANY, ready but not issued = SQ_WAIT_INST_ANY, "
                  "each over SQ_WAVE_CYCLES; MFMA co-issue = SQ_VALU_MFMA_COEXEC_CYCLES over "
                  "SQ_VALU_MFMA_BUSY_CYCLES.", "",
              "| launch | issuing | waiting (dependency, barrier) | ready, not issued | MFMA co-issue with other VALU | "
              "LDS command FIFO full (cycles per active cycle per CU) |",
              "|---|---|---|---|---|---|"]
        for i, d in enumerate(ds):
            c = dict(d["ctr"])
            for e in extra:
                for k, v in e[i]["ctr"].items():
                    c.setdefault(k, v)
            wc = c.get("SQ_WAVE_CYCLES")
            if not wc or "SQ_ACTIVE_INST_ANY" not in c or "SQ_WAIT_INST_ANY" not in c:
                continue
            active = c["GRBM_GUI_ACTIVE"] / GRBM_INSTANCES
            co = c.get("SQ_VALU_MFMA_COEXEC_CYCLES", float("nan")) / c["SQ_VALU_MFMA_BUSY_CYCLES"]
            ff = c.get("SQ_LDS_CMD_FIFO_FULL", float("nan")) / (active * 256)
            L.append(f"| {i + 1} | {c['SQ_ACTIVE_INST_ANY'] / wc:.3f} | {c['SQ_WAIT_ANY'] / wc:.3f} | "
                     f"{c['SQ_WAIT_INST_ANY'] / wc:.3f} | {co:.3f} | {ff:.4f} |")
    with open(args.md or os.path.join(ROOT, "profiles", "gemm_bf16_4096_counters.md"), "w") as f:
        f.write("\n".join(L) + "\n")
    print(json.dumps({"written": args.md or "profiles/gemm_bf16_4096_counters.md", "launches": len(ds)}))


STRESSOR_KERNELS = ("stream_stressor<", "strided_stressor<", "cache_stressor", "lds_stressor<", "valu_stressor<",
                    "valu64_stressor<", "mfma_stressor<", "chase_stressor<", "empty_wg")


def run_suite_counter_summary(args):
    """Per-stressor counters of `--config suite-counters` from four
    rocprofv3 --pmc databases (--dbs A B F W: caches and GRBM, SQ, FETCH_SIZE,
    WRITE_SIZE): writes profiles/stressor_counters.md."""
    dbs = dict(zip("ABFW", args.dbs))
    per = None
    for key, db in dbs.items():
        ds = [d for d in _pmc_dispatches(db) if d["name"].startswith(STRESSOR_KERNELS)]
        if len(ds) != len(SUITE_LABELS):
            raise SystemExit(f"{db}: {len(ds)} stressor dispatches, expected {len(SUITE_LABELS)}")
        if per is None:
            per = [{"kernel": d["name"], "grid": d["grid"], "wg": d["wg"]} for d in ds]
        for i, d in enumerate(ds):
            per[i].update(d["ctr"])
    with open(os.path.join(ROOT, "profiles", "hbm_triad_n2e30_counters.json")) as f:
        cal = json.load(f)["calibration_copy_1GiB"]
    ff, wf = cal["fetch_factor"], cal["write_factor"]
    g = lambda c, *names: next((c[n] for n in names if n in c), float("nan"))
    L = ["# Hardware counters per stressor (one fixed-work launch each, MI355X)", "",
         "Commands (repository root; one counter set per run), then the summary:", "", "```"]
    L += args.cmd + [" ".join(["python3 bench.py --config suite-counter-summary --dbs"] + list(args.dbs)), "```", "",
                     "Derived columns: active us = GRBM_GUI_ACTIVE / 8 XCDs / 2.4 GHz; L2 hit = TCC_HIT / (TCC_HIT "
                     "+ TCC_MISS); vL1D hit = 1 - TCP_TCC_READ_REQ / TCP_TOTAL_CACHE_ACCESSES; VALU busy = 4 x "
                     "SQ_INSTS_VALU / SIMD-cycles; MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES / SIMD-cycles (SIMD-cycles "
                     "= active cycles x 1024 SIMDs); LDS instr/CU/clk = SQ_INSTS_LDS / (active cycles x 256 CUs); "
                     f"read / written past L2 = FETCH_SIZE x {ff:.4f} / WRITE_SIZE x {wf:.4f} KiB (the 1 GiB copy "
                     "calibration of hbm_triad_n2e30_counters.md): traffic between the L2s and the memory side, "
                     "served by the Infinity Cache or HBM; TB/s over the active time.", "",
                     "| stressor | kernel | active us | L2 hit | L2 requests | vL1D hit | vL1D accesses | LDS instr | "
                     "LDS bank conflicts | VALU busy | MFMA busy | waves | LDS instr/CU/clk | read past L2 GB | "
                     "written past L2 GB | past L2 TB/s |",
                     "|---|---|---|---|---|---|---|---|---|---|---|---|---|---|---|---|"]
    for (name, label), c in zip(SUITE_LABELS, per):
        cyc = g(c, "GRBM_GUI_ACTIVE") / GRBM_INSTANCES
        us = cyc / 2.4e3
        hit, miss = g(c, "TCC_HIT_sum", "TCC_HIT"), g(c, "TCC_MISS_sum", "TCC_MISS")
        tcp = g(c, "TCP_TOTAL_CACHE_ACCESSES_sum", "TCP_TOTAL_CACHE_ACCESSES")
        tcp_miss = g(c, "TCP_TCC_READ_REQ_sum", "TCP_TCC_READ_REQ")
        simd = cyc * 1024
        rd = g(c, "FETCH_SIZE") * 1024 * ff / 1e9
        wr = g(c, "WRITE_SIZE") * 1024 * wf / 1e9
        L.append(f"| {label} | `{c['kernel']}` | {us:.1f} | {hit / (hit + miss):.3f} | {hit + miss:.3g} | "
                 f"{1 - tcp_miss / tcp if tcp else float('nan'):.4f} | {tcp:.3g} | {g(c, 'SQ_INSTS_LDS'):.3g} | "
                 f"{g(c, 'SQ_LDS_BANK_CONFLICT'):.0f} | {4 * g(c, 'SQ_INSTS_VALU') / simd:.2f} | "
                 f"{g(c, 'SQ_VALU_MFMA_BUSY_CYCLES') / simd:.2f} | {g(c, 'SQ_WAVES'):.0f} | "
                 f"{g(c, 'SQ_INSTS_LDS') / (cyc * 256):.3f} | {rd:.3f} | {wr:.3f} | {(rd + wr) / (us * 1e-6) / 1e3:.2f} |")
    out = os.path.join(ROOT, "profiles", "stressor_counters.md")
    with open(out, "w") as f:
        f.write("\n".join(L) + "\n")
    print(json.dumps({"written": out}))


# LDS stressor forms of `--config lds-counters`, in launch order:
# (access, vector width in words, stride in vectors, passes, work-groups of 16 waves per CU)
LDS_COUNTER_FORMS = [("copy", 4, 1, 10, 1), ("load", 4, 1, 20, 1), ("load", 4, 1, 20, 2), ("copy", 4, 1, 10, 2),
                     ("load", 2, 1, 10, 1), ("load", 1, 1, 5, 1),
                     ("copy", 1, 1, 4, 1), ("copy", 1, 2, 4, 1), ("copy", 1, 4, 2, 1), ("copy", 1, 8, 2, 1),
                     ("copy", 1, 16, 1, 1), ("copy", 1, 32, 1, 1), ("copy", 1, 64, 1, 1), ("load", 1, 2, 4, 1),
                     ("load", 1, 32, 1, 1)]


def run_lds_counters(args):
    """Short run for hardware-counter passes on the LDS stressor: each form
    of LDS_COUNTER_FORMS once on every CU (16 waves per CU, fixed work)."""
    import torch
    import synth
    from paper_2501_16909_amd import coloc
    dev = torch.device("cuda:0")
    ctx = coloc.Context(0)
    w = torch.from_numpy(synth.u32(synth.seed_for(1, synth.BUF_LDS), 8192).view(np.int32)).to(dev)
    rows = []
    for access, vec, stride, passes, wgs in LDS_COUNTER_FORMS:
        rep = ctx.stressor("lds", 1.0, src0=w, vec=vec, knob=stride, passes=passes, wg_per_cu=wgs,
                           access=coloc.LDS_ACCESS[access]).stop()
        rows.append({"access": access, "vec": vec, "stride": stride, "waves_per_cu": 16 * wgs,
                     "tb_s": round(rep.achieved / 1e12, 2), "pct_of_peak": round(rep.pct_of_peak, 1)})
        log(f"lds {access} vec {vec} stride {stride} {16 * wgs} waves/CU: {rep.achieved / 1e12:.2f} TB/s "
            f"({rep.pct_of_peak:.1f} %)")
    ctx.close()
    print(json.dumps({"counters_run": "lds stressor forms", "forms": rows}), flush=True)


def run_lds_counter_summary(args):
    """LDS counters of `--config lds-counters` from the rocprofv3 --pmc
    databases given with --dbs: writes profiles/lds_stride_counters.md."""
    per = [dict() for _ in LDS_COUNTER_FORMS]
    for db in args.dbs:
        ds = [d for d in _pmc_dispatches(db) if d["name"].startswith("lds_stressor<")]
        if len(ds) != len(LDS_COUNTER_FORMS):
            raise SystemExit(f"{db}: {len(ds)} LDS dispatches, expected {len(LDS_COUNTER_FORMS)}")
        for i, d in enumerate(ds):
            per[i].update(d["ctr"])
    cus = 256
    L = ["# LDS stressor: bank conflicts, LDS activity and bytes per clock (hardware counters)", "",
         "Commands (repository root, one MI355X; one counter set per run), then the summary:", "", "```"]
    L += args.cmd + [" ".join(["python3 bench.py --config lds-counter-summary --dbs"] + list(args.dbs)), "```", "",
                     "`bench.py --config lds-counters` runs each form below once on all 256 CUs (one or two "
                     "work-groups of 16 waves per CU, 64 KiB of LDS each, fixed work).  A stride of s vectors "
                     "sends lane l to vector (l s + k) mod (8192 / width) on step k.", "",
                     "Bytes per clock per CU = (SQ_INSTS_LDS_LOAD_BANDWIDTH + SQ_INSTS_LDS_STORE_BANDWIDTH) x 64 "
                     "/ (GRBM_GUI_ACTIVE / 8) / 256; LDS active = SQ_LDS_IDX_ACTIVE / (GRBM_GUI_ACTIVE / 8) / 256; "
                     "bank-conflict share = SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE; instruction issue = "
                     "clocks per LDS instruction per CU.", "",
                     "| form | width (words) | stride | waves/CU | B/clk/CU loaded | B/clk/CU stored | LDS active | "
                     "bank-conflict share | address-conflict share | clocks per LDS instruction |",
                     "|---|---|---|---|---|---|---|---|---|---|"]
    for (access, vec, stride, _, wgs), c in zip(LDS_COUNTER_FORMS, per):
        cyc = c["GRBM_GUI_ACTIVE"] / GRBM_INSTANCES
        ld = c.get("SQ_INSTS_LDS_LOAD_BANDWIDTH", 0.0) * 64 / cyc / cus
        stb = c.get("SQ_INSTS_LDS_STORE_BANDWIDTH", 0.0) * 64 / cyc / cus
        act = c.get("SQ_LDS_IDX_ACTIVE", float("nan")) / cyc / cus
        bank = c.get("SQ_LDS_BANK_CONFLICT", float("nan")) / c.get("SQ_LDS_IDX_ACTIVE", float("nan"))
        addr = c.get("SQ_LDS_ADDR_CONFLICT", float("nan")) / c.get("SQ_LDS_IDX_ACTIVE", float("nan"))
        ipc = cyc * cus / c["SQ_INSTS_LDS"] if c.get("SQ_INSTS_LDS") else float("nan")
        L.append(f"| {access} | {vec} | {stride} | {16 * wgs} | {ld:.1f} | {stb:.1f} | {100 * act:.1f} % | {100 * bank:.1f} % | "
                 f"{100 * addr:.1f} % | {ipc:.2f} |")
    out = os.path.join(ROOT, "profiles", "lds_stride_counters.md")
    with open(out, "w") as f:
        f.write("\n".join(L) + "\n")
    print(json.dumps({"written": out}))


def run_counters(args):
    """Short run for hardware-counter passes: the HBM stressor over N = 2^30
    (one pass per launch) twice, its read-only, copy and write-only mixes
    once each, then a plain 1 GiB device-to-device copy
    twice as the calibration kernel of known traffic (1 GiB read, 1 GiB
    written)."""
    import torch
    import synth
    from paper_2501_16909_amd import coloc
    dev = torch.device("cuda:0")
    ctx = coloc.Context(0)
    n = 1 << 30
    b = torch.empty(n, dtype=torch.float32, device=dev)
    c, a = torch.empty_like(b), torch.empty_like(b)
    synth.device_fill_uniform_f32(b.data_ptr(), n, synth.seed_for(1, synth.BUF_B))
    synth.device_fill_uniform_f32(c.data_ptr(), n, synth.seed_for(1, synth.BUF_C))
    torch.cuda.synchronize()
    for _ in range(2):
        rep = ctx.stressor("hbm", 1.0, src0=b, src1=c, dst=a, n=n, passes=1).stop()
        log(f"hbm stressor: {rep.units / rep.kernel_ns:.0f} GB/s")
    for mix, ops in (("read", dict(src0=b, src1=c)), ("copy", dict(src0=b, dst=a)), ("write", dict(dst=a))):
        rep = ctx.stressor("hbm", 1.0, n=n, passes=1, knob=coloc.HBM_MIX[mix], **ops).stop()
        log(f"hbm stressor, {mix} mix: {rep.units / rep.kernel_ns:.0f} GB/s")
    src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    ctx.close()
    print(json.dumps({"counters_run": "hbm_triad_n2e30 x2, read/copy/write mixes x1, copy 1GiB x2"}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="suite", choices=["suite", "sweep", "precision", "serve", "counters", "suite-counters",
                             "pollution", "bandwidth", "ilp", "pairs", "ldsstride", "estimator", "decode",
                             "queues", "hbm_mix", "gemm-counters", "counter-summary", "trace-summary",
                             "lds-counters", "lds-counter-summary", "suite-counter-summary",
                             "gemm-counter-summary", "hbm-references", "reference-summary",
                             "chase-latency", "serve-background"])
    ap.add_argument("--dbs", nargs="+", default=[], help="summaries: rocprofv3 databases to read")
    ap.add_argument("--cmd", nargs="+", default=[], help="summaries: the commands that made the databases")
    ap.add_argument("--md", default=None, help="trace-summary: markdown file to write")
    ap.add_argument("--title", default="Kernel trace", help="trace-summary: heading")
    ap.add_argument("--top", type=int, default=0, help="trace-summary: rows kept (0 = all)")
    ap.add_argument("--window-ms", type=float, default=0.0,
                    help="trace-summary: list launches longer than this and the kernels inside them")
    ap.add_argument("--bench-json", default=None, help="trace-summary: the benchmark line of the traced run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick", action="store_true",
                    help="suite: the timed stressor suite only (no sensitivity, precision or serving blocks)")
    ap.add_argument("--suite-reps", type=int, default=5,
                    help="suite: counterbalanced pairs per cell of the sensitivity block")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="suite: length of the 200/s serving trace (the 1000/s trace is a sixth of it)")
    ap.add_argument("--stressor-warmup", type=int, default=0,
                    help="suite: untimed launches of each stressor right before its timed one")
    ap.add_argument("--out", default=None, help="also write the JSON line(s) to this file")
    ap.add_argument("--reps", type=int, default=10, help="sweep / precision: repetitions per cell")
    ap.add_argument("--deadline-ms", type=int, default=200,
                    help="sweep / precision / serve: stressor deadline per colocated run")
    ap.add_argument("--rates", type=float, nargs="+", default=[200.0, 1000.0, 3000.0],
                    help="serve: arrival rates per second")
    ap.add_argument("--seconds", type=float, default=2.0, help="serve: trace length")
    ap.add_argument("--bound", type=float, default=1.5, help="serve: p99 slowdown bound")
    ap.add_argument("--duty", type=int, default=50,
                    help="serve-background: duty cycle (percent) of the background HBM stressor")
    ap.add_argument("--background-mix", default="triad", choices=["triad", "read"],
                    help="serve-background: traffic mix of the background HBM stressor")
    ap.add_argument("--profiles", default=None, help="serve: sensitivity profiles (JSON)")
    ap.add_argument("--batch", type=int, default=1, help="decode: sequences per step (1..8)")
    ap.add_argument("--contexts", type=int, default=6, help="queues: fresh contexts (queue orders) to try")
    ap.add_argument("--profile-runs", type=int, default=1,
                    help="estimator / serve: profile measurements per curve, combined point-wise by the median")
    ap.add_argument("--profile-axis", default="duty", choices=["cu", "duty"],
                    help="serve: intensity axis of measured profiles (CU fraction or duty cycle)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the colocation "
                                   "harness measures interference inside a single device",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.config == "suite":
        run_suite(args)
    elif args.config == "counters":
        run_counters(args)
    elif args.config == "suite-counters":
        run_suite_counters(args)
    elif args.config == "sweep":
        run_sweep(args)
    elif args.config == "precision":
        run_precision(args)
    elif args.config == "serve":
        run_serve(args)
    elif args.config == "pollution":
        run_pollution(args)
    elif args.config == "bandwidth":
        run_bandwidth(args)
    elif args.config == "ilp":
        run_ilp(args)
    elif args.config == "pairs":
        run_pairs(args)
    elif args.config == "ldsstride":
        run_ldsstride(args)
    elif args.config == "estimator":
        run_estimator(args)
    elif args.config == "decode":
        run_decode(args)
    elif args.config == "queues":
        run_queues(args)
    elif args.config == "hbm_mix":
        run_hbm_mix(args)
    elif args.config == "gemm-counters":
        run_gemm_counters(args)
    elif args.config == "counter-summary":
        run_counter_summary(args)
    elif args.config == "trace-summary":
        run_trace_summary(args)
    elif args.config == "lds-counters":
        run_lds_counters(args)
    elif args.config == "lds-counter-summary":
        run_lds_counter_summary(args)
    elif args.config == "suite-counter-summary":
        run_suite_counter_summary(args)
    elif args.config == "gemm-counter-summary":
        run_gemm_counter_summary(args)
    elif args.config == "hbm-references":
        run_hbm_references(args)
    elif args.config == "chase-latency":
        run_chase_latency(args)
    elif args.config == "reference-summary":
        run_reference_summary(args)
    elif args.config == "serve-background":
        run_serve_background(args)


if __name__ == "__main__":
    main()
