"""Python binding of libcoloc.so (include/coloc.h): argument marshalling only.

Every step runs in the library's HIP kernels; torch supplies device memory
and streams.  Loading fails loudly when the library is not built.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcoloc.so")

RESOURCES = ["hbm", "l2", "mall", "vl1d", "lds", "valu_f32", "mfma_f32", "mfma_bf16",
             "mfma_fp8", "ptrchase", "dispatch", "occupancy", "valu_f64"]
RES = {name: i for i, name in enumerate(RESOURCES)}
DTYPES = {"f32": 0, "bf16": 1, "fp8": 2}
# HBM stressor traffic mixes (its `knob`): CI_HBM_TRIAD / READ / COPY / WRITE
HBM_MIX = {"triad": 1, "read": 2, "copy": 3, "write": 4}
LDS_ACCESS = {"copy": 0, "load": 1}
VICTIMS = {"triad": 0, "gemm": 1, "gemv": 2}
POLICIES = {"naive": 0, "usher": 1, "sensitivity": 2}
STATUS = {0: "CI_OK", 1: "CI_ERR_INVALID_ARG", 2: "CI_ERR_HIP", 3: "CI_ERR_OOM",
          4: "CI_ERR_TIMEOUT", 5: "CI_ERR_UNSUPPORTED", 6: "CI_ERR_BUSY", 7: "CI_ERR_DRAIN"}
NPOINTS = 5
NRES = len(RESOURCES)


class CiError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class DeviceInfo(C.Structure):
    _fields_ = [("device", C.c_int), ("num_cus", C.c_int), ("num_xcds", C.c_int),
                ("wave_size", C.c_int), ("clock_khz", C.c_int), ("wall_clock_khz", C.c_int),
                ("lds_bytes_per_cu", C.c_uint64), ("l2_bytes_per_xcd", C.c_uint64),
                ("hbm_bytes", C.c_uint64), ("arch", C.c_char * 64),
                ("peak", C.c_double * NRES)]


class WgRecord(C.Structure):
    _fields_ = [("t_start", C.c_uint64), ("t_end", C.c_uint64), ("work", C.c_uint64),
                ("check", C.c_uint64), ("loc", C.c_uint32), ("flags", C.c_uint32),
                ("pad", C.c_uint64)]


class StressorOpts(C.Structure):
    _fields_ = [("src0", C.c_void_p), ("src1", C.c_void_p), ("dst", C.c_void_p),
                ("n", C.c_uint64), ("wg_per_cu", C.c_uint32), ("threads", C.c_uint32),
                ("knob", C.c_uint32), ("vec", C.c_uint32), ("passes", C.c_uint64),
                ("iters", C.c_uint64), ("fa", C.c_float), ("fb", C.c_float),
                ("deadline_ms", C.c_uint32), ("duty", C.c_uint32), ("chunk", C.c_uint32),
                ("access", C.c_uint32)]


class StressorReport(C.Structure):
    _fields_ = [("resource", C.c_int), ("ncu", C.c_int), ("grid", C.c_uint32),
                ("wg_reported", C.c_uint32), ("t_first_start", C.c_uint64),
                ("t_last_start", C.c_uint64), ("t_first_end", C.c_uint64),
                ("t_last_end", C.c_uint64), ("window_ns", C.c_double), ("kernel_ns", C.c_double),
                ("work", C.c_uint64), ("units", C.c_double), ("achieved", C.c_double),
                ("pct_of_peak", C.c_double), ("checksum", C.c_uint64), ("timed_out", C.c_int),
                ("distinct_cus", C.c_int)]


class VictimDesc(C.Structure):
    _fields_ = [("kind", C.c_int), ("dtype", C.c_int), ("m", C.c_uint64), ("n", C.c_uint64),
                ("k", C.c_uint64), ("a", C.c_void_p), ("b", C.c_void_p), ("out", C.c_void_p),
                ("scale_a", C.c_float), ("scale_b", C.c_float), ("passes", C.c_uint32),
                ("copies", C.c_uint32), ("flags", C.c_uint32), ("reserved", C.c_uint32)]


class VictimResult(C.Structure):
    _fields_ = [("time_ns", C.c_double), ("checksum_bits", C.c_uint64), ("sum_f64", C.c_double),
                ("t_begin", C.c_uint64), ("t_end", C.c_uint64)]


MEASURE_NO_QUEUE_CHECK = 1


class MeasureOpts(C.Structure):
    _fields_ = [("reps", C.c_uint32), ("warmups", C.c_uint32), ("placement", C.c_int),
                ("deadline_ms", C.c_uint32), ("flags", C.c_uint32),
                ("rep_alone_ns", C.POINTER(C.c_double)), ("rep_col_ns", C.POINTER(C.c_double))]


class Cell(C.Structure):
    _fields_ = [("resource", C.c_int), ("intensity", C.c_float), ("ncu", C.c_int),
                ("slowdown", C.c_double), ("slowdown_p10", C.c_double),
                ("slowdown_p90", C.c_double), ("t_alone_ns", C.c_double),
                ("t_col_ns", C.c_double), ("stressor_achieved", C.c_double),
                ("stressor_pct_peak", C.c_double), ("window_covered", C.c_int),
                ("output_equal", C.c_int), ("timed_out", C.c_int), ("reps", C.c_int),
                ("slowdown_ci_lo", C.c_double), ("slowdown_ci_hi", C.c_double),
                ("queue_unresolved", C.c_int)]


class Profile(C.Structure):
    _fields_ = [("kind", C.c_int), ("sens", (C.c_float * NPOINTS) * NRES),
                ("press", C.c_float * NRES), ("occ", C.c_float),
                ("sens_hbm_read", C.c_float * NPOINTS), ("press_hbm_read", C.c_float),
                ("hbm_write_frac", C.c_float)]


class Request(C.Structure):
    _fields_ = [("arrival_s", C.c_double), ("kind", C.c_int), ("dtype", C.c_int),
                ("m", C.c_uint64), ("n", C.c_uint64), ("k", C.c_uint64), ("seed", C.c_uint64),
                ("out_copy", C.c_void_p)]


class Policy(C.Structure):
    _fields_ = [("kind", C.c_int), ("bound", C.c_double), ("hbm_budget", C.c_uint64),
                ("slots", C.c_int), ("profiles", C.POINTER(Profile)), ("nprofiles", C.c_int),
                ("background", C.POINTER(Profile))]


class Served(C.Structure):
    _fields_ = [("arrival_s", C.c_double), ("admit_s", C.c_double), ("end_s", C.c_double),
                ("service_ns", C.c_double), ("checksum_bits", C.c_uint64), ("sum_f64", C.c_double),
                ("slot", C.c_int), ("status", C.c_int)]


DECODE_KERNELS = ["qkv", "attn", "attn_combine", "oproj", "gate_up", "down", "lm_head"]
NDK = len(DECODE_KERNELS)
DECODE_KERNEL_TIMES, DECODE_GRAPH = 1, 2
GEMV_EPILOGUES = {"plain": 0, "silu": 1, "rope": 2}
NOALLOC_PART_BYTES = 16 << 20   # CI_NOALLOC_PART_BYTES: static scratch for partial results


class DecodeConfig(C.Structure):
    _fields_ = [("hidden", C.c_uint32), ("n_q", C.c_uint32), ("n_kv", C.c_uint32),
                ("head_dim", C.c_uint32), ("ffn", C.c_uint32), ("vocab", C.c_uint32),
                ("layers", C.c_uint32), ("batch", C.c_uint32), ("max_ctx", C.c_uint32),
                ("eps", C.c_float), ("rope_base", C.c_float)]


class DecodeLayout(C.Structure):
    _fields_ = [("g_attn", C.c_uint64), ("w_qkv", C.c_uint64), ("w_o", C.c_uint64),
                ("g_mlp", C.c_uint64), ("w_gu", C.c_uint64), ("w_down", C.c_uint64),
                ("layer_stride", C.c_uint64), ("g_final", C.c_uint64), ("w_lm", C.c_uint64),
                ("weight_elems", C.c_uint64), ("cache_elems", C.c_uint64),
                ("workspace_bytes", C.c_uint64), ("attn_part_bytes", C.c_uint64)]


class DecodeDesc(C.Structure):
    _fields_ = [("cfg", DecodeConfig), ("weights", C.c_void_p), ("k_cache", C.c_void_p),
                ("v_cache", C.c_void_p), ("pos", C.POINTER(C.c_int32)), ("x_in", C.c_void_p),
                ("x_out", C.c_void_p), ("logits", C.c_void_p), ("work", C.c_void_p),
                ("flags", C.c_uint32), ("reserved", C.c_uint32)]


class GemvArgs(C.Structure):
    _fields_ = [("w", C.c_void_p), ("rows", C.c_uint32), ("k", C.c_uint32), ("batch", C.c_uint32),
                ("epilogue", C.c_int), ("v", C.c_void_p), ("x", C.c_void_p), ("g", C.c_void_p),
                ("eps", C.c_float), ("res", C.c_void_p), ("out", C.c_void_p), ("h", C.c_void_p),
                ("pos", C.POINTER(C.c_int32)), ("n_q", C.c_uint32), ("n_kv", C.c_uint32),
                ("head_dim", C.c_uint32), ("max_ctx", C.c_uint32), ("rope_base", C.c_float),
                ("q_out", C.c_void_p), ("k_cache", C.c_void_p), ("v_cache", C.c_void_p)]


class DecodeResult(C.Structure):
    _fields_ = [("step_ns", C.c_double), ("kernel_ns", C.c_double * NDK),
                ("checksum_bits", C.c_uint64), ("sum_f64", C.c_double),
                ("t_begin", C.c_uint64), ("t_end", C.c_uint64)]


class DecodeCell(C.Structure):
    _fields_ = [("resource", C.c_int), ("intensity", C.c_float), ("duty", C.c_uint32),
                ("ncu", C.c_int), ("step_alone_p50", C.c_double), ("step_alone_p90", C.c_double),
                ("step_col_p50", C.c_double), ("step_col_p90", C.c_double),
                ("kernel_alone_ns", C.c_double * NDK), ("kernel_col_ns", C.c_double * NDK),
                ("stressor_achieved", C.c_double), ("stressor_pct_peak", C.c_double),
                ("window_covered", C.c_int), ("output_equal", C.c_int), ("timed_out", C.c_int),
                ("reps", C.c_int), ("queue_unresolved", C.c_int)]


EXPORTS = {
    "ci_init": ([C.c_int, C.POINTER(C.c_void_p)], C.c_int),
    "ci_shutdown": ([C.c_void_p], C.c_int),
    "ci_last_error": ([], C.c_char_p),
    "ci_device_info": ([C.c_void_p, C.POINTER(DeviceInfo)], C.c_int),
    "ci_peak_for": ([C.c_void_p, C.c_int, C.POINTER(C.c_double)], C.c_int),
    "ci_cu_mask": ([C.c_void_p, C.c_float, C.c_int, C.POINTER(C.c_uint32), C.POINTER(C.c_int)], C.c_int),
    "ci_probe_placement": ([C.c_void_p, C.POINTER(C.c_uint32), C.c_uint32, C.c_void_p], C.c_int),
    "ci_queue_stats": ([C.c_void_p, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)],
                       C.c_int),
    "ci_bootstrap_slowdown": ([C.POINTER(C.c_double), C.c_uint32, C.POINTER(C.c_double), C.c_uint32,
                               C.c_uint32, C.c_uint64, C.POINTER(C.c_double), C.POINTER(C.c_double)],
                              C.c_int),
    "ci_workspace_size": ([C.c_int, C.c_float, C.POINTER(StressorOpts), C.POINTER(C.c_size_t)], C.c_int),
    "stressor_launch": ([C.c_void_p, C.c_int, C.c_float, C.c_void_p, C.POINTER(StressorOpts),
                         C.c_void_p, C.c_size_t, C.POINTER(C.c_void_p)], C.c_int),
    "stressor_stop": ([C.c_void_p, C.POINTER(StressorReport)], C.c_int),
    "ci_read_records": ([C.c_void_p, C.c_void_p, C.c_uint32, C.POINTER(WgRecord)], C.c_int),
    "victim_run": ([C.c_void_p, C.POINTER(VictimDesc), C.c_void_p, C.POINTER(VictimResult)], C.c_int),
    "victim_enqueue": ([C.c_void_p, C.POINTER(VictimDesc), C.c_void_p, C.c_uint32], C.c_int),
    "ci_stamp": ([C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "ci_checksum_f32": ([C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p, C.POINTER(C.c_uint64),
                         C.POINTER(C.c_double)], C.c_int),
    "ci_quantize": ([C.c_void_p, C.c_void_p, C.c_uint64, C.c_int, C.c_void_p, C.POINTER(C.c_float),
                     C.c_void_p], C.c_int),
    "ci_mfma_probe": ([C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32,
                       C.c_void_p], C.c_int),
    "measure_sensitivity": ([C.c_void_p, C.POINTER(VictimDesc), C.POINTER(C.c_int),
                             C.POINTER(StressorOpts), C.c_int, C.POINTER(C.c_float), C.c_int,
                             C.POINTER(MeasureOpts), C.c_void_p, C.c_size_t, C.c_void_p,
                             C.POINTER(Cell)], C.c_int),
    "serve_run": ([C.c_void_p, C.POINTER(Request), C.c_int, C.POINTER(Policy), C.POINTER(Served)], C.c_int),
    "serve_run_background": ([C.c_void_p, C.POINTER(Request), C.c_int, C.POINTER(Policy), C.c_int, C.c_float,
                              C.POINTER(StressorOpts), C.c_void_p, C.c_size_t, C.POINTER(Served),
                              C.POINTER(StressorReport)], C.c_int),
    "ci_admit": ([C.POINTER(Policy), C.POINTER(C.c_int), C.c_int, C.c_int, C.c_uint64, C.c_uint64,
                  C.POINTER(C.c_int)], C.c_int),
    "ci_predict_slowdown": ([C.POINTER(Profile), C.POINTER(C.POINTER(Profile)), C.c_int,
                             C.POINTER(C.c_double)], C.c_int),
    "decode_layout": ([C.POINTER(DecodeConfig), C.POINTER(DecodeLayout)], C.c_int),
    "decode_step": ([C.c_void_p, C.POINTER(DecodeDesc), C.c_void_p, C.POINTER(DecodeResult)], C.c_int),
    "measure_decode": ([C.c_void_p, C.POINTER(DecodeDesc), C.POINTER(C.c_int), C.POINTER(StressorOpts),
                        C.c_int, C.POINTER(C.c_float), C.c_int, C.POINTER(MeasureOpts), C.c_void_p,
                        C.c_size_t, C.c_void_p, C.POINTER(DecodeCell)], C.c_int),
    "ci_rmsnorm_bf16": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32, C.c_uint32, C.c_float,
                         C.c_void_p, C.c_void_p], C.c_int),
    "ci_gemv_bf16_rows": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32,
                           C.c_uint32, C.c_uint32, C.c_void_p], C.c_int),
    "ci_rope_append": ([C.c_void_p, C.c_void_p, C.POINTER(C.c_int32), C.c_uint32, C.c_uint32, C.c_uint32,
                        C.c_uint32, C.c_uint32, C.c_float, C.c_void_p, C.c_void_p, C.c_void_p,
                        C.c_void_p], C.c_int),
    "ci_attention_decode": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_int32),
                             C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_void_p,
                             C.c_size_t, C.c_void_p, C.c_void_p], C.c_int),
    "ci_attention_decode_noalloc": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_int32),
                                     C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_void_p,
                                     C.c_void_p], C.c_int),
    "ci_silu_mul_bf16": ([C.c_void_p, C.c_void_p, C.c_uint32, C.c_uint32, C.c_void_p, C.c_void_p], C.c_int),
    "ci_fused_gemv": ([C.c_void_p, C.POINTER(GemvArgs), C.c_void_p], C.c_int),
}

_LIB = None
# Stressors running anywhere in this process (any context): while one runs,
# nothing here touches torch's legacy null stream (see Context._sync_torch).
_RUNNING: set = set()


def load_library(path: str = LIB_PATH):
    """Load libcoloc.so and declare every exported entry point."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built: run python -m paper_2501_16909_amd.build "
                               "(the device library has no fallback)")
        lib = C.CDLL(path)
        for name, (args, res) in EXPORTS.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _LIB = lib
    return _LIB


def _check(st: int):
    if st != 0:
        msg = load_library().ci_last_error()
        raise CiError(st, msg.decode() if msg else "")


def _ptr(t) -> int | None:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream_handle(stream) -> int | None:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


@dataclass
class Report:
    resource: str
    ncu: int
    grid: int
    wg_reported: int
    t_first_start: int
    t_last_start: int
    t_first_end: int
    t_last_end: int
    window_ns: float
    kernel_ns: float
    work: int
    units: float
    achieved: float
    pct_of_peak: float
    checksum: int
    timed_out: bool
    distinct_cus: int
    status: int = 0


def _report(r: StressorReport, st: int) -> Report:
    return Report(RESOURCES[r.resource], r.ncu, r.grid, r.wg_reported, r.t_first_start,
                  r.t_last_start, r.t_first_end, r.t_last_end, r.window_ns, r.kernel_ns, r.work,
                  r.units, r.achieved, r.pct_of_peak, r.checksum, bool(r.timed_out), r.distinct_cus,
                  st)


def bootstrap_slowdown(alone, col, resamples: int = 1000, seed: int = 0) -> tuple:
    """(lo, hi): the library's percentile-bootstrap 95 % interval of
    median(col) / median(alone) (host computation)."""
    a = np.ascontiguousarray(alone, dtype=np.float64)
    c = np.ascontiguousarray(col, dtype=np.float64)
    lo, hi = C.c_double(), C.c_double()
    _check(load_library().ci_bootstrap_slowdown(a.ctypes.data_as(C.POINTER(C.c_double)), a.size,
                                                c.ctypes.data_as(C.POINTER(C.c_double)), c.size,
                                                int(resamples), int(seed), C.byref(lo), C.byref(hi)))
    return lo.value, hi.value


def make_opts(**kw) -> StressorOpts:
    o = StressorOpts()
    for k, v in kw.items():
        if k in ("src0", "src1", "dst"):
            setattr(o, k, _ptr(v))
        else:
            setattr(o, k, v)
    return o


class Stressor:
    """A running stressor; use as a context manager or call stop()."""

    def __init__(self, ctx: "Context", resource: str, intensity: float, stream=None,
                 ws=None, keep=(), **opts):
        import torch
        self.ctx = ctx
        self.resource = resource
        self.opts = make_opts(**opts)
        self._keep = keep  # tensors that must outlive the kernel
        lib = load_library()
        need = C.c_size_t()
        _check(lib.ci_workspace_size(RES[resource], 1.0, C.byref(self.opts), C.byref(need)))
        if ws is None:
            ws = torch.empty(max(int(need.value), 256), dtype=torch.uint8, device=ctx.device)
        self.ws = ws
        self.stream = stream
        h = C.c_void_p()
        _check(lib.stressor_launch(ctx.handle, RES[resource], float(intensity),
                                   _stream_handle(stream), C.byref(self.opts), _ptr(ws),
                                   ws.numel(), C.byref(h)))
        self.h = h
        self.report: Report | None = None
        ctx._active = self
        _RUNNING.add(id(self))

    def stop(self, raise_on_timeout: bool = True) -> Report:
        if self.h is None:
            return self.report
        rep = StressorReport()
        st = load_library().stressor_stop(self.h, C.byref(rep))
        self.h = None
        self.ctx._active = None
        _RUNNING.discard(id(self))
        self.report = _report(rep, st)
        if st != 0 and not (st == 4 and not raise_on_timeout):
            _check(st)
        return self.report

    def records(self) -> np.ndarray:
        """Per-work-group records (valid after stop())."""
        g = self.report.grid if self.report else 0
        arr = (WgRecord * max(g, 1))()
        _check(load_library().ci_read_records(self.ctx.handle, _ptr(self.ws), g, arr))
        dt = np.dtype([("t_start", "<u8"), ("t_end", "<u8"), ("work", "<u8"), ("check", "<u8"),
                       ("loc", "<u4"), ("flags", "<u4"), ("pad", "<u8")])
        return np.frombuffer(bytes(arr), dtype=dt, count=g).copy()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.stop(raise_on_timeout=exc[0] is None)
        return False


@dataclass
class VictimOutcome:
    time_ns: float
    checksum_bits: int
    sum_f64: float
    t_begin: int
    t_end: int


class Context:
    def __init__(self, device: int = 0):
        import torch
        lib = load_library()
        h = C.c_void_p()
        _check(lib.ci_init(int(device), C.byref(h)))
        self.handle = h
        self.device = torch.device("cuda", device)
        info = DeviceInfo()
        _check(lib.ci_device_info(h, C.byref(info)))
        self.info = info
        self.stream = torch.cuda.Stream(device=self.device)
        self._active = None

    def close(self):
        if self.handle:
            _check(load_library().ci_shutdown(self.handle))
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    # -------------------------------------------------------------- info
    def peak(self, resource: str) -> float:
        v = C.c_double()
        _check(load_library().ci_peak_for(self.handle, RES[resource], C.byref(v)))
        return v.value

    def cu_mask(self, intensity: float, complement: bool = False):
        m = (C.c_uint32 * 8)()
        n = C.c_int()
        _check(load_library().ci_cu_mask(self.handle, float(intensity), int(complement), m, C.byref(n)))
        return list(m), n.value

    def probe_placement(self, mask, nwg: int) -> np.ndarray:
        import torch
        out = torch.zeros(nwg, dtype=torch.int32, device=self.device)
        torch.cuda.synchronize(self.device)
        mp = (C.c_uint32 * 8)(*mask) if mask is not None else None
        _check(load_library().ci_probe_placement(self.handle, mp, nwg, _ptr(out)))
        return out.cpu().numpy().view(np.uint32)

    def queue_stats(self) -> dict:
        """Queue-pair check counters (see ci_queue_stats in coloc.h)."""
        v = [C.c_uint32() for _ in range(3)]
        _check(load_library().ci_queue_stats(self.handle, *[C.byref(x) for x in v]))
        return {"checks": v[0].value, "replaced": v[1].value, "unresolved": v[2].value}

    # ---------------------------------------------------------- stressors
    def _sync_torch(self):
        """Finish torch's queued work before a library call.  Skipped while any
        stressor runs in this process: torch's default stream is the legacy
        null stream, and synchronising it would also wait for every CU-masked
        stressor stream."""
        import torch
        if not _RUNNING:
            torch.cuda.current_stream(self.device).synchronize()

    def stressor(self, resource: str, intensity: float, stream=None, ws=None, **opts) -> Stressor:
        self._sync_torch()
        keep = tuple(v for k, v in opts.items() if k in ("src0", "src1", "dst") and v is not None)
        return Stressor(self, resource, intensity, stream if stream is not None else self.stream,
                        ws=ws, keep=keep, **opts)

    # ------------------------------------------------------------ victims
    def victim_run(self, desc: VictimDesc, stream=None) -> VictimOutcome:
        self._sync_torch()
        r = VictimResult()
        s = stream if stream is not None else self.stream
        _check(load_library().victim_run(self.handle, C.byref(desc), _stream_handle(s), C.byref(r)))
        return VictimOutcome(r.time_ns, r.checksum_bits, r.sum_f64, r.t_begin, r.t_end)

    def victim_enqueue(self, desc: VictimDesc, stream, count: int):
        """Queue `count` launches of the victim on `stream` without waiting."""
        self._sync_torch()
        _check(load_library().victim_enqueue(self.handle, C.byref(desc), _stream_handle(stream), int(count)))

    def stamp(self, slot, stream):
        """Enqueue a device wall-clock stamp into slot (a one-element int64
        device tensor, or a view of one) on stream; returns at once."""
        _check(load_library().ci_stamp(self.handle, _ptr(slot), _stream_handle(stream)))

    @staticmethod
    def triad_desc(b, c, a, passes: int = 1, in_kernel: bool = False) -> VictimDesc:
        """in_kernel: the passes run inside one launch (CI_VICTIM_TRIAD_IN_KERNEL)."""
        d = VictimDesc()
        d.kind, d.dtype, d.n = 0, 0, b.numel()
        d.flags = 1 if in_kernel else 0
        d.a, d.b, d.out = _ptr(b), _ptr(c), _ptr(a)
        d.passes, d.copies, d.scale_a, d.scale_b = passes, 1, 1.0, 1.0
        d._keep = (b, c, a)   # the descriptor holds raw pointers: keep the tensors alive
        return d

    @staticmethod
    def gemm_desc(A, B, Cm, dtype: str, m: int, n: int, k: int, scale_a=1.0, scale_b=1.0) -> VictimDesc:
        d = VictimDesc()
        d.kind, d.dtype, d.m, d.n, d.k = 1, DTYPES[dtype], m, n, k
        d.a, d.b, d.out = _ptr(A), _ptr(B), _ptr(Cm)
        d.scale_a, d.scale_b, d.passes, d.copies = float(scale_a), float(scale_b), 1, 1
        d._keep = (A, B, Cm)
        return d

    @staticmethod
    def gemv_desc(W, x, y, n: int, k: int, copies: int = 1) -> VictimDesc:
        d = VictimDesc()
        d.kind, d.dtype, d.n, d.k = 2, 1, n, k
        d.a, d.b, d.out = _ptr(W), _ptr(x), _ptr(y)
        d.copies, d.passes, d.scale_a, d.scale_b = copies, 1, 1.0, 1.0
        d._keep = (W, x, y)
        return d

    def victim_triad(self, b, c, a, passes: int = 1, stream=None, in_kernel: bool = False) -> VictimOutcome:
        return self.victim_run(self.triad_desc(b, c, a, passes, in_kernel), stream)

    def checksum(self, x) -> tuple:
        self._sync_torch()
        bits, s = C.c_uint64(), C.c_double()
        _check(load_library().ci_checksum_f32(self.handle, _ptr(x), x.numel(),
                                              _stream_handle(self.stream), C.byref(bits), C.byref(s)))
        return bits.value, s.value

    def quantize(self, x, dtype: str):
        """(codes tensor, scale): BF16 (uint16 codes viewed as int16) or FP8 (uint8)."""
        import torch
        self._sync_torch()
        if dtype == "bf16":
            out = torch.empty(x.shape, dtype=torch.int16, device=x.device)
        elif dtype == "fp8":
            out = torch.empty(x.shape, dtype=torch.uint8, device=x.device)
        else:
            raise ValueError(dtype)
        sc = C.c_float()
        _check(load_library().ci_quantize(self.handle, _ptr(x), x.numel(), DTYPES[dtype], _ptr(out),
                                          C.byref(sc), _stream_handle(self.stream)))
        return out, sc.value

    def mfma_probe(self, dtype: str, a, b, c, d):
        """ci_mfma_probe: one matrix-core instruction per tile, d = a b + c (device tensors,
        tiles contiguous; a, b as the dtype's codes)."""
        self._sync_torch()
        ntiles = c.numel() // 1024
        _check(load_library().ci_mfma_probe(self.handle, DTYPES[dtype], _ptr(a), _ptr(b), _ptr(c), _ptr(d),
                                            ntiles, _stream_handle(self.stream)))

    # -------------------------------------------------------- sensitivity
    def measure_sensitivity(self, desc: VictimDesc, resources, opts_list, intensities,
                            reps: int = 20, warmups: int = 3, placement: str = "shared",
                            deadline_ms: int = 2000, ws=None, queue_check: bool = True):
        import torch
        self._sync_torch()
        nr, nx = len(resources), len(intensities)
        rs = (C.c_int * nr)(*[RES[r] for r in resources])
        so = (StressorOpts * nr)(*[make_opts(**o) for o in opts_list])
        xs = (C.c_float * nx)(*[float(x) for x in intensities])
        per_rep = nr * nx * reps
        rep_a = (C.c_double * per_rep)()
        rep_c = (C.c_double * per_rep)()
        mo = MeasureOpts(reps, warmups, 1 if placement == "disjoint" else 0, deadline_ms,
                         0 if queue_check else MEASURE_NO_QUEUE_CHECK, rep_a, rep_c)
        need = 256
        for i in range(nr):
            b = C.c_size_t()
            _check(load_library().ci_workspace_size(rs[i], 1.0, C.byref(so[i]), C.byref(b)))
            need = max(need, int(b.value))
        if ws is None:
            ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        cells = (Cell * (nr * nx))()
        _check(load_library().measure_sensitivity(self.handle, C.byref(desc), rs, so, nr, xs, nx,
                                                  C.byref(mo), _ptr(ws), ws.numel(),
                                                  _stream_handle(self.stream), cells))
        out = []
        for q, c in enumerate(cells):
            out.append({f: getattr(c, f) for f, _ in Cell._fields_})
            out[-1]["resource"] = RESOURCES[c.resource]
            out[-1]["rep_alone_ns"] = list(rep_a[q * reps:(q + 1) * reps])
            out[-1]["rep_col_ns"] = list(rep_c[q * reps:(q + 1) * reps])
        return out

    # ------------------------------------------------------------- decode
    @staticmethod
    def decode_layout(cfg: dict) -> DecodeLayout:
        c = DecodeConfig(**{f: cfg[f] for f, _ in DecodeConfig._fields_})
        out = DecodeLayout()
        _check(load_library().decode_layout(C.byref(c), C.byref(out)))
        return out

    def decode_step(self, model: "DecodeModel") -> dict:
        self._sync_torch()
        r = DecodeResult()
        _check(load_library().decode_step(self.handle, C.byref(model.desc), _stream_handle(self.stream),
                                          C.byref(r)))
        return {"step_ns": r.step_ns, "kernel_ns": dict(zip(DECODE_KERNELS, list(r.kernel_ns))),
                "checksum_bits": r.checksum_bits, "sum_f64": r.sum_f64, "t_begin": r.t_begin,
                "t_end": r.t_end}

    def measure_decode(self, model: "DecodeModel", resources, opts_list, intensities, reps: int = 10,
                       warmups: int = 2, placement: str = "shared", deadline_ms: int = 2000, ws=None,
                       queue_check: bool = True):
        import torch
        self._sync_torch()
        nr, nx = len(resources), len(intensities)
        rs = (C.c_int * nr)(*[RES[r] for r in resources])
        so = (StressorOpts * nr)(*[make_opts(**o) for o in opts_list])
        xs = (C.c_float * nx)(*[float(x) for x in intensities])
        mo = MeasureOpts(reps, warmups, 1 if placement == "disjoint" else 0, deadline_ms,
                         0 if queue_check else MEASURE_NO_QUEUE_CHECK)
        if ws is None:
            need = 256
            for i in range(nr):
                b = C.c_size_t()
                _check(load_library().ci_workspace_size(rs[i], 1.0, C.byref(so[i]), C.byref(b)))
                need = max(need, int(b.value))
            ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        cells = (DecodeCell * (nr * nx))()
        _check(load_library().measure_decode(self.handle, C.byref(model.desc), rs, so, nr, xs, nx,
                                             C.byref(mo), _ptr(ws), ws.numel(),
                                             _stream_handle(self.stream), cells))
        out = []
        for c in cells:
            d = {f: getattr(c, f) for f, _ in DecodeCell._fields_ if not f.startswith("kernel_")}
            d["resource"] = RESOURCES[c.resource]
            d["kernel_alone_ns"] = dict(zip(DECODE_KERNELS, list(c.kernel_alone_ns)))
            d["kernel_col_ns"] = dict(zip(DECODE_KERNELS, list(c.kernel_col_ns)))
            out.append(d)
        return out

    def rmsnorm_bf16(self, x, g, eps: float, y=None):
        import torch
        self._sync_torch()
        rows, n = x.shape
        if y is None:
            y = torch.empty((rows, n), dtype=torch.int16, device=x.device)
        _check(load_library().ci_rmsnorm_bf16(self.handle, _ptr(x), _ptr(g), rows, n, float(eps), _ptr(y),
                                              _stream_handle(self.stream)))
        return y

    def gemv_bf16_rows(self, w, v, res=None, out=None):
        """out[b] = res[b] + w @ v[b]; w rows x k BF16 codes, v batch x k."""
        import torch
        self._sync_torch()
        rows, k = w.shape
        batch = v.shape[0]
        if out is None:
            out = torch.empty((batch, rows), dtype=torch.float32, device=w.device)
        _check(load_library().ci_gemv_bf16_rows(self.handle, _ptr(w), _ptr(v), _ptr(res), _ptr(out), rows, k,
                                                batch, _stream_handle(self.stream)))
        return out

    def rope_append(self, qkv, pos, n_q: int, n_kv: int, head_dim: int, max_ctx: int, rope_base: float,
                    q_out, k_cache, v_cache):
        self._sync_torch()
        batch = len(pos)
        p = (C.c_int32 * batch)(*[int(v) for v in pos])
        _check(load_library().ci_rope_append(self.handle, _ptr(qkv), p, batch, n_q, n_kv, head_dim, max_ctx,
                                             float(rope_base), _ptr(q_out), _ptr(k_cache), _ptr(v_cache),
                                             _stream_handle(self.stream)))

    def attention_decode(self, q, k_cache, v_cache, pos, n_q: int, n_kv: int, head_dim: int, max_ctx: int,
                         out=None):
        import torch
        self._sync_torch()
        batch = len(pos)
        lay = self.decode_layout(dict(hidden=8, n_q=n_q, n_kv=n_kv, head_dim=head_dim, ffn=8, vocab=0,
                                      layers=1, batch=batch, max_ctx=max_ctx, eps=0.0, rope_base=1.0))
        part = torch.empty(max(int(lay.attn_part_bytes), 16), dtype=torch.uint8, device=q.device)
        if out is None:
            out = torch.empty((batch, n_q * head_dim), dtype=torch.int16, device=q.device)
        p = (C.c_int32 * batch)(*[int(v) for v in pos])
        _check(load_library().ci_attention_decode(self.handle, _ptr(q), _ptr(k_cache), _ptr(v_cache), p, batch,
                                                  n_q, n_kv, head_dim, max_ctx, _ptr(part), part.numel(),
                                                  _ptr(out), _stream_handle(self.stream)))
        return out

    def attention_decode_noalloc(self, q, k_cache, v_cache, pos, n_q: int, n_kv: int, head_dim: int,
                                 max_ctx: int, out):
        """attention_decode working in the library's static device scratch:
        the call allocates nothing; the caller passes the output."""
        self._sync_torch()
        batch = len(pos)
        p = (C.c_int32 * batch)(*[int(v) for v in pos])
        _check(load_library().ci_attention_decode_noalloc(self.handle, _ptr(q), _ptr(k_cache), _ptr(v_cache), p,
                                                          batch, n_q, n_kv, head_dim, max_ctx, _ptr(out),
                                                          _stream_handle(self.stream)))
        return out

    def fused_gemv(self, w, epilogue: str = "plain", v=None, x=None, g=None, eps: float = 0.0, res=None,
                   out=None, h=None, pos=None, n_q: int = 0, n_kv: int = 0, head_dim: int = 0,
                   max_ctx: int = 0, rope_base: float = 1.0, q_out=None, k_cache=None, v_cache=None):
        """The decode step's GEMV with its fused prologue (RMS norm of x when
        v is None) and epilogue ("plain", "silu", "rope")."""
        self._sync_torch()
        rows, k = w.shape
        batch = (v if v is not None else x).shape[0]
        a = GemvArgs()
        a.w, a.rows, a.k, a.batch, a.epilogue = _ptr(w), rows, k, batch, GEMV_EPILOGUES[epilogue]
        a.v, a.x, a.g, a.eps = _ptr(v), _ptr(x), _ptr(g), float(eps)
        a.res, a.out, a.h = _ptr(res), _ptr(out), _ptr(h)
        keep = None
        if pos is not None:
            keep = (C.c_int32 * batch)(*[int(p) for p in pos])
            a.pos = C.cast(keep, C.POINTER(C.c_int32))
        a.n_q, a.n_kv, a.head_dim, a.max_ctx, a.rope_base = n_q, n_kv, head_dim, max_ctx, float(rope_base)
        a.q_out, a.k_cache, a.v_cache = _ptr(q_out), _ptr(k_cache), _ptr(v_cache)
        _check(load_library().ci_fused_gemv(self.handle, C.byref(a), _stream_handle(self.stream)))

    def silu_mul_bf16(self, gu, ffn: int, h=None):
        import torch
        self._sync_torch()
        batch = gu.shape[0]
        if h is None:
            h = torch.empty((batch, ffn), dtype=torch.int16, device=gu.device)
        _check(load_library().ci_silu_mul_bf16(self.handle, _ptr(gu), batch, ffn, _ptr(h),
                                               _stream_handle(self.stream)))
        return h

    # ------------------------------------------------------------ serving
    @staticmethod
    def _serve_args(requests, policy, bound, hbm_budget, slots, profiles, background):
        n = len(requests)
        tr = (Request * max(n, 1))()
        for i, q in enumerate(requests):
            tr[i] = Request(q["arrival_s"], VICTIMS[q["kind"]], DTYPES[q.get("dtype", "f32")],
                            q.get("m", 0), q.get("n", 0), q.get("k", 0), q["seed"],
                            _ptr(q["out_copy"]) if q.get("out_copy") is not None else None)
        profs = make_profiles(profiles or {})
        bg = make_load_profile(background) if background is not None else None
        pol = Policy(POLICIES[policy], bound, hbm_budget, slots,
                     C.cast(profs, C.POINTER(Profile)) if len(profs) else None, len(profs),
                     C.pointer(bg) if bg is not None else None)
        pol._keep = (profs, bg)   # the policy holds raw pointers into these
        return tr, n, pol, (Served * max(n, 1))()

    def serve(self, requests, policy: str = "naive", bound: float = 1.5, hbm_budget: int = 8 << 30,
              slots: int = 4, profiles=None, background=None):
        """serve_run.  background: the load of a co-runner present throughout,
        as a profile dict ("press", "occ", read/write fields), for the
        admission rules (serve_loaded also runs one)."""
        self._sync_torch()
        tr, n, pol, out = self._serve_args(requests, policy, bound, hbm_budget, slots, profiles, background)
        _check(load_library().serve_run(self.handle, tr, n, C.byref(pol), out))
        return [{f: getattr(out[i], f) for f, _ in Served._fields_} for i in range(n)]

    def serve_loaded(self, requests, resource: str, intensity: float, ws=None, policy: str = "naive",
                     bound: float = 1.5, hbm_budget: int = 8 << 30, slots: int = 4, profiles=None,
                     background=None, **opts):
        """serve_run_background: serve `requests` while stressor `resource`
        runs at CU fraction `intensity` with stressor options `opts` (its
        operands and knobs, passes 0).  background: the stressor's load
        profile for the admission rules (None: admission does not see it).
        Returns (served records, the stressor's Report); raises CiError on
        any error, also when the stressor stopped on its deadline."""
        import torch
        self._sync_torch()
        tr, n, pol, out = self._serve_args(requests, policy, bound, hbm_budget, slots, profiles, background)
        o = make_opts(**opts)
        if ws is None:
            need = C.c_size_t()
            _check(load_library().ci_workspace_size(RES[resource], 1.0, C.byref(o), C.byref(need)))
            ws = torch.empty(max(int(need.value), 256), dtype=torch.uint8, device=self.device)
        rep = StressorReport()
        st = load_library().serve_run_background(self.handle, tr, n, C.byref(pol), RES[resource],
                                                 float(intensity), C.byref(o), _ptr(ws), ws.numel(), out,
                                                 C.byref(rep))
        _check(st)
        return [{f: getattr(out[i], f) for f, _ in Served._fields_} for i in range(n)], _report(rep, st)


class DecodeModel:
    """Device buffers of one synthetic decode step: BF16 weight arena and
    KV caches drawn from the seeded streams of synth.decode_tensor_specs,
    the FP32 residual-stream input, outputs and workspace."""

    def __init__(self, ctx: Context, cfg: dict, pos, seed: int, flags: int = DECODE_KERNEL_TIMES):
        import torch
        import synth
        self.cfg = dict(cfg)
        self.layout = lay = ctx.decode_layout(self.cfg)
        dev = ctx.device
        lib = load_library()
        self.weights = torch.empty(int(lay.weight_elems), dtype=torch.int16, device=dev)
        self.k_cache = torch.empty(int(lay.cache_elems), dtype=torch.int16, device=dev)
        self.v_cache = torch.empty(int(lay.cache_elems), dtype=torch.int16, device=dev)
        b, hid = cfg["batch"], cfg["hidden"]
        self.x_in = torch.empty((b, hid), dtype=torch.float32, device=dev)
        self.x_out = torch.empty((b, hid), dtype=torch.float32, device=dev)
        self.logits = torch.empty((b, max(cfg["vocab"], 1)), dtype=torch.float32, device=dev)
        self.work = torch.empty(max(int(lay.workspace_bytes), 256), dtype=torch.uint8, device=dev)
        specs = synth.decode_tensor_specs(self.cfg, seed)
        biggest = max(n for _, _, _, n, _, _ in specs)
        stage = torch.empty(max(biggest, 1), dtype=torch.float32, device=dev)
        torch.cuda.synchronize(dev)
        stream = _stream_handle(ctx.stream)
        for name, layer, sd, n, scale, offset in specs:
            if n == 0:
                continue
            if name == "x_in":
                synth.device_fill_affine_f32(_ptr(self.x_in), n, sd, scale, offset, stream=stream)
                continue
            if name in ("k_cache", "v_cache"):
                dst = _ptr(getattr(self, name))
            else:
                off = getattr(lay, name) + (layer * lay.layer_stride if layer >= 0 else 0)
                dst = _ptr(self.weights) + 2 * int(off)
            synth.device_fill_affine_f32(_ptr(stage), n, sd, scale, offset, stream=stream)
            sc = C.c_float()
            _check(lib.ci_quantize(ctx.handle, _ptr(stage), n, DTYPES["bf16"], dst, C.byref(sc), stream))
        ctx.stream.synchronize()
        del stage
        self.flags = flags
        self.set_positions(pos)

    def set_positions(self, pos):
        self.pos = (C.c_int32 * self.cfg["batch"])(*[int(p) for p in pos])
        d = DecodeDesc()
        d.cfg = DecodeConfig(**{f: self.cfg[f] for f, _ in DecodeConfig._fields_})
        d.weights, d.k_cache, d.v_cache = _ptr(self.weights), _ptr(self.k_cache), _ptr(self.v_cache)
        d.pos = C.cast(self.pos, C.POINTER(C.c_int32))
        d.x_in, d.x_out = _ptr(self.x_in), _ptr(self.x_out)
        d.logits = _ptr(self.logits) if self.cfg["vocab"] else None
        d.work = _ptr(self.work)
        d.flags = self.flags
        self.desc = d

    def set_flags(self, flags: int):
        self.flags = flags
        self.desc.flags = flags

    def tensor(self, name: str, layer: int = -1):
        """View of one weight tensor of the arena (BF16 codes as int16)."""
        lay = self.layout
        spec = {s[0]: s[3] for s in __import__("synth").decode_tensor_specs(self.cfg, 0) if s[1] in (0, -1)}
        off = getattr(lay, name) + (layer * lay.layer_stride if layer >= 0 else 0)
        return self.weights[int(off):int(off) + spec[name]]


def _fill_profile(dst: Profile, p: dict):
    for r in range(NRES):
        for j in range(NPOINTS):
            dst.sens[r][j] = 1.0
        dst.press[r] = 0.0
    for rname, curve in p.get("sens", {}).items():
        for j, v in enumerate(curve):
            dst.sens[RES[rname]][j] = float(v)
    for rname, v in p.get("press", {}).items():
        dst.press[RES[rname]] = float(v)
    dst.occ = float(p.get("occ", 0.0))
    for j, v in enumerate(p.get("sens_hbm_read") or [0.0] * NPOINTS):
        dst.sens_hbm_read[j] = float(v)
    dst.press_hbm_read = float(p.get("press_hbm_read", 0.0))
    dst.hbm_write_frac = float(p.get("hbm_write_frac", 1.0))


def make_profiles(profiles: dict):
    """profiles: {kind name: {"sens": {res: [5 slowdowns]}, "press": {res: p}, "occ": o}}, and
    optionally "sens_hbm_read" (5 slowdowns against the read-only HBM mix), "press_hbm_read"
    and "hbm_write_frac" (read/write-aware HBM pricing, see ci_predict_slowdown)."""
    arr = (Profile * max(len(profiles), 1))()
    for i, (kind, p) in enumerate(profiles.items()):
        arr[i].kind = VICTIMS[kind]
        _fill_profile(arr[i], p)
    if not profiles:
        return (Profile * 0)()
    return arr


def make_load_profile(p: dict) -> Profile:
    """A background load for ci_policy_t.background: "press" per resource,
    "occ", and the optional read/write fields, as in make_profiles (its kind
    and curves are not read)."""
    out = Profile()
    out.kind = -1
    _fill_profile(out, p)
    return out


def predict_slowdown(profiles: dict, victim: str, corunners) -> float:
    """ci_predict_slowdown of kind `victim` beside co-runners: kind names in
    profiles, or load profile dicts (make_load_profile) such as a background."""
    names = list(profiles)
    arr = make_profiles(profiles)
    loads = [make_load_profile(k) for k in corunners if isinstance(k, dict)]
    it = iter(loads)
    co = (C.POINTER(Profile) * max(len(corunners), 1))(
        *[C.pointer(next(it)) if isinstance(k, dict) else C.pointer(arr[names.index(k)]) for k in corunners])
    out = C.c_double()
    _check(load_library().ci_predict_slowdown(C.byref(arr[names.index(victim)]), co, len(corunners),
                                              C.byref(out)))
    return out.value


def admit(policy: str, profiles: dict, running_kinds, cand_kind: str, cand_bytes: int,
          free_bytes: int, bound: float = 1.5, slots: int = 4, background=None) -> bool:
    """ci_admit; background: a load profile dict present throughout (make_load_profile)."""
    profs = make_profiles(profiles)
    bg = make_load_profile(background) if background is not None else None
    pol = Policy(POLICIES[policy], bound, 1 << 40, slots,
                 C.cast(profs, C.POINTER(Profile)) if len(profs) else None, len(profs),
                 C.pointer(bg) if bg is not None else None)
    rk = (C.c_int * max(len(running_kinds), 1))(*[VICTIMS[k] for k in running_kinds])
    out = C.c_int()
    _check(load_library().ci_admit(C.byref(pol), rk, len(running_kinds), VICTIMS[cand_kind],
                                   cand_bytes, free_bytes, C.byref(out)))
    return bool(out.value)
