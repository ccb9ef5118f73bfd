"""CPU oracle of the colocation suite.

TEST INFRASTRUCTURE ONLY: plain, slow and obviously correct.  Only the tests,
``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the device library
(``paper_2501_16909_amd``) and never imports it.

Bit-level steps (two-rounding triad, FMA chains, pointer walk, quantizers,
exact summation) live in ``coloc_oracle.c`` and are loaded with ctypes;
dense products use numpy in FP64 as a library step.  Each function names
the passage of the paper (Elvinger et al., SoCC'25) or the workload
definition it follows.

Parity status per function (pins are in tests/test_oracle_pins.py; the decode
submodule's in tests/test_oracle_decode.py):
  triad_f32, triad_f32_threads, bitsum_u32, sum_f32_exact  pinned
  hbm_read_checksum, hbm_copy, hbm_write_pattern  pinned
  fma_chain_f32 / valu_outputs .................. pinned
  dmul_chain_f64 / valu64_outputs ............... pinned
  chase_u32, is_single_cycle .................... pinned
  cache_wg_expected, lds_wave_pass_sum .......... pinned
  f32_to_bf16, f32_to_e4m3, quantize_fp8 ........ pinned
  gemm_f64, gemv_f64, mfma_tile_expected ........ pinned
  slowdown, pct_of_peak ......................... pinned (paper Table 1 values)
  bootstrap_slowdown_ci ......................... pinned (closed-form resampling law)
  accumulation_bound ............................ pinned (brute force, toy format)
  e4m3_nominal_exponent, mfma_fp8_error_bound ... pinned (hand case, exact model)
  predicted_slowdown, predicted_slowdown_rw, admit  pinned
  simulate_admission, FirstFitArena ............. pinned
  decode (submodule: synthetic decode step) ..... pinned
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "coloc_oracle.c")
_SO = os.path.join(_HERE, "libcoloc_oracle.so")
_LIB = None

_F32P = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_U32P = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_U64P = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
_U16P = np.ctypeslib.ndpointer(dtype=np.uint16, flags="C_CONTIGUOUS")
_U8P = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")


def build_oracle(force: bool = False) -> str:
    """Compile coloc_oracle.c with gcc (no fused multiply-add contraction)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-pthread",
                               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _lib():
    global _LIB
    if _LIB is None:
        lib = ctypes.CDLL(build_oracle())
        lib.or_triad_f32.argtypes = [_F32P, _F32P, _F32P, ctypes.c_uint64]
        lib.or_triad_f32_mt.argtypes = [_F32P, _F32P, _F32P, ctypes.c_uint64, ctypes.c_int]
        lib.or_triad_f32_mt.restype = ctypes.c_int
        lib.or_bitsum_u32.argtypes = [_U32P, ctypes.c_uint64]
        lib.or_bitsum_u32.restype = ctypes.c_uint64
        lib.or_sum_u32_mod32.argtypes = [_U32P, ctypes.c_uint64, ctypes.c_uint64]
        lib.or_sum_u32_mod32.restype = ctypes.c_uint32
        lib.or_sum_f32_exact.argtypes = [_F32P, ctypes.c_uint64]
        lib.or_sum_f32_exact.restype = ctypes.c_double
        lib.or_fma_chain_f32.argtypes = [_F32P, ctypes.c_uint64, ctypes.c_float, ctypes.c_float,
                                         ctypes.c_uint64, _F32P]
        lib.or_dmul_chain.argtypes = [np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS"),
                                      ctypes.c_uint64, ctypes.c_double, ctypes.c_uint64,
                                      np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")]
        lib.or_chase_u32.argtypes = [_U32P, ctypes.c_uint64, _U64P, ctypes.c_uint64,
                                     ctypes.c_uint64, _U32P]
        lib.or_is_single_cycle.argtypes = [_U32P, ctypes.c_uint64]
        lib.or_is_single_cycle.restype = ctypes.c_int
        lib.or_lds_wave_pass_sum.argtypes = [_U32P, ctypes.c_uint32, ctypes.c_uint32,
                                             ctypes.c_uint32]
        lib.or_lds_wave_pass_sum.restype = ctypes.c_uint32
        lib.or_f32_to_bf16.argtypes = [_F32P, ctypes.c_uint64, _U16P]
        lib.or_e4m3_decode.argtypes = [ctypes.c_uint8]
        lib.or_e4m3_decode.restype = ctypes.c_double
        lib.or_f32_to_e4m3.argtypes = [_F32P, ctypes.c_uint64, _U8P]
        _LIB = lib
    return _LIB


def _f32(x):
    return np.ascontiguousarray(x, dtype=np.float32)


# --------------------------------------------------------------------------
# Triad: copy-style bandwidth kernel.  The paper's copy kernel repeatedly
# copies an input array to an output array (Section 3, Pitfall 2; Section
# 4.3); the workload here is the STREAM triad a = b + 3c in FP32, which moves
# two input streams and one output stream.  Repeated passes rewrite the same
# values, so the output does not depend on how many passes ran.
# --------------------------------------------------------------------------
def triad_f32(b, c) -> np.ndarray:
    b, c = _f32(b), _f32(c)
    if b.shape != c.shape:
        raise ValueError("b and c must have the same shape")
    a = np.empty_like(b)
    _lib().or_triad_f32(b.ravel(), c.ravel(), a.ravel(), b.size)
    return a


def triad_f32_threads(b, c, threads: int, out=None) -> tuple:
    """triad_f32 split over `threads` host threads (contiguous shares; the
    result is the same for any count).  Returns (a, threads that ran)."""
    b, c = _f32(b), _f32(c)
    if b.shape != c.shape:
        raise ValueError("b and c must have the same shape")
    a = np.empty_like(b) if out is None else out
    ran = _lib().or_triad_f32_mt(b.ravel(), c.ravel(), a.ravel(), b.size, int(threads))
    return a, int(ran)


def bitsum_u32(x) -> int:
    """Sum of the 32-bit patterns of x modulo 2**64 (order independent)."""
    w = np.ascontiguousarray(x).view(np.uint32).ravel()
    return int(_lib().or_bitsum_u32(w, w.size))


def sum_f32_exact(x) -> float:
    """Exact sum of FP32 values rounded to FP64."""
    x = _f32(x).ravel()
    return float(_lib().or_sum_f32_exact(x, x.size))


def rel_err_sum(device_sum: float, x) -> float:
    """Relative error of a device FP sum of x against the exact sum; falls
    back to a normwise error (divide by sum |x|) when the sum nearly cancels
    (|sum| < 1e-3 * sum|x|)."""
    exact = sum_f32_exact(x)
    absum = sum_f32_exact(np.abs(_f32(x)))
    denom = abs(exact) if abs(exact) >= 1e-3 * absum else absum
    if denom == 0.0:
        return abs(device_sum - exact)
    return abs(device_sum - exact) / denom


# --------------------------------------------------------------------------
# HBM traffic mixes.  The bandwidth stressor of Section 3 (Pitfall 2) and
# Section 4.3 streams large arrays; besides the triad it can read only, copy,
# or write only, which sets the read/write proportion of the DRAM traffic.
# Per element (4-byte words): read-only folds b[i] + c[i] into a checksum
# mod 2**32 (once per pass), copy stores b's bits, write-only stores
# lo32(i) * 0x9E3779B1 mod 2**32.
# --------------------------------------------------------------------------
HBM_MIXES = {"triad": 1, "read": 2, "copy": 3, "write": 4}
WRITE_MULTIPLIER = 0x9E3779B1


def hbm_bytes_per_element(mix: str) -> int:
    """Bytes a mix moves per element: triad 2 reads + 1 write, read-only and
    copy two streams, write-only one."""
    return {"triad": 12, "read": 8, "copy": 8, "write": 4}[mix]


def hbm_read_checksum(b, c, passes: int) -> int:
    """passes x sum over i of (b[i] + c[i]) as uint32 words, mod 2**32."""
    s = (region_sum_u32(np.ascontiguousarray(b).view(np.uint32))
         + region_sum_u32(np.ascontiguousarray(c).view(np.uint32))) % (1 << 32)
    return (int(passes) * s) % (1 << 32)


def hbm_copy(b) -> np.ndarray:
    """The copy mix's output: b's 32-bit words, NaN payloads included."""
    return np.ascontiguousarray(b).view(np.uint32).copy()


def hbm_write_pattern(n: int, first: int = 0) -> np.ndarray:
    """Words the write-only mix stores at indices first .. first + n - 1."""
    i = (np.arange(first, first + n, dtype=np.uint64) & np.uint64(0xFFFFFFFF))
    return ((i * np.uint64(WRITE_MULTIPLIER)) & np.uint64(0xFFFFFFFF)).astype(np.uint32)


# --------------------------------------------------------------------------
# Cache working-set loops (vL1D, L2, Infinity Cache).  Every work-group sums
# the 32-bit words of its region once per pass; the region is the same for
# all work-groups.  Expected per-work-group checksum after P passes:
# P * sum(region) mod 2**32.  Pass counts are run-until-stop on the device,
# so the check uses the pass count each work-group reports.
# --------------------------------------------------------------------------
def region_sum_u32(words, lo: int = 0, hi: int | None = None) -> int:
    w = np.ascontiguousarray(words, dtype=np.uint32).ravel()
    hi = w.size if hi is None else hi
    return int(_lib().or_sum_u32_mod32(w, lo, hi))


def cache_wg_expected(region_words, passes) -> np.ndarray:
    s = region_sum_u32(region_words)
    p = np.asarray(passes, dtype=np.uint64)
    return ((p * np.uint64(s)) & np.uint64(0xFFFFFFFF)).astype(np.uint32)


# --------------------------------------------------------------------------
# LDS loop (shared-memory bandwidth / bank-conflict kernel, Section 4.4.1).
# The window holds `nvec` vectors of `vw` words; at step k lane l reads
# vector (l*stride + k) mod nvec (and writes it back to the twin window).
# --------------------------------------------------------------------------
def lds_wave_pass_sum(window_words, vw: int, stride: int) -> int:
    w = np.ascontiguousarray(window_words, dtype=np.uint32).ravel()
    if w.size % vw:
        raise ValueError("window size must be a multiple of the vector width")
    return int(_lib().or_lds_wave_pass_sum(w, w.size // vw, vw, stride))


def lds_wg_expected(window_words, vw: int, stride: int, waves: int, passes) -> np.ndarray:
    s = lds_wave_pass_sum(window_words, vw, stride)
    p = np.asarray(passes, dtype=np.uint64)
    return ((p * np.uint64(waves) * np.uint64(s)) & np.uint64(0xFFFFFFFF)).astype(np.uint32)


# --------------------------------------------------------------------------
# VALU chain (compute kernel, Section 3 and Sections 4.4.2-4.4.3): each lane
# runs `ilp` independent chains x <- fma(x, a, b).  Start values:
# x0(t, c) = ((t mod 1024) + c + 1) * 2**-10 for global thread t, chain c.
# --------------------------------------------------------------------------
def fma_chain_f32(x0, a: float, b: float, steps: int) -> np.ndarray:
    x0 = _f32(x0).ravel()
    out = np.empty_like(x0)
    _lib().or_fma_chain_f32(x0, x0.size, np.float32(a), np.float32(b), int(steps), out)
    return out


def valu_start_values(threads, ilp: int) -> np.ndarray:
    t = np.asarray(threads, dtype=np.uint64)
    c = np.arange(ilp, dtype=np.uint64)
    k = (t[:, None] % np.uint64(1024)) + c[None, :] + np.uint64(1)
    return (k.astype(np.float64) * 2.0 ** -10).astype(np.float32)


def valu_outputs(threads, ilp: int, a: float, b: float, steps: int) -> np.ndarray:
    """Final chain values, shape (len(threads), ilp)."""
    x0 = valu_start_values(threads, ilp)
    return fma_chain_f32(x0.ravel(), a, b, steps).reshape(x0.shape)


def dmul_chain_f64(x0, a: float, steps: int) -> np.ndarray:
    """FP64 pipeline chain (Section 4.4.3): x <- x * a, `steps` times."""
    x0 = np.ascontiguousarray(x0, dtype=np.float64).ravel()
    out = np.empty_like(x0)
    _lib().or_dmul_chain(x0, x0.size, float(a), int(steps), out)
    return out


def valu64_outputs(threads, ilp: int, a: float, steps: int) -> np.ndarray:
    """FP64 stressor outputs, shape (len(threads), ilp); start values as for
    the FP32 chains, x0(t, c) = ((t mod 1024) + c + 1) * 2**-10."""
    t = np.asarray(threads, dtype=np.uint64)
    c = np.arange(ilp, dtype=np.uint64)
    k = (t[:, None] % np.uint64(1024)) + c[None, :] + np.uint64(1)
    x0 = k.astype(np.float64) * 2.0 ** -10
    return dmul_chain_f64(x0.ravel(), a, steps).reshape(x0.shape)


# --------------------------------------------------------------------------
# Pointer chase: i <- next[i], `hops` times from each start.
# --------------------------------------------------------------------------
def chase_u32(nxt, starts, hops: int) -> np.ndarray:
    nxt = np.ascontiguousarray(nxt, dtype=np.uint32)
    st = np.ascontiguousarray(starts, dtype=np.uint64)
    end = np.empty(st.size, dtype=np.uint32)
    _lib().or_chase_u32(nxt, nxt.size, st, st.size, int(hops), end)
    return end


def chase_starts(nchains: int, n: int) -> np.ndarray:
    """Evenly spaced starts: chain q of Q begins at floor(q * n / Q)."""
    q = np.arange(nchains, dtype=np.uint64)
    return (q * np.uint64(n)) // np.uint64(nchains)


def is_single_cycle(nxt) -> bool:
    nxt = np.ascontiguousarray(nxt, dtype=np.uint32)
    r = _lib().or_is_single_cycle(nxt, nxt.size)
    if r < 0:
        raise MemoryError("oracle could not allocate the visit map")
    return bool(r)


# --------------------------------------------------------------------------
# Quantizers (precision extension).
# --------------------------------------------------------------------------
def f32_to_bf16(x) -> np.ndarray:
    """Round-to-nearest-even FP32 -> BF16 codes (uint16)."""
    x = _f32(x)
    out = np.empty(x.shape, dtype=np.uint16)
    _lib().or_f32_to_bf16(x.ravel(), x.size, out.reshape(-1))
    return out


def bf16_to_f64(codes) -> np.ndarray:
    c = np.ascontiguousarray(codes, dtype=np.uint16)
    return (c.astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)


def e4m3_decode(code: int) -> float:
    return float(_lib().or_e4m3_decode(int(code) & 0xFF))


def e4m3_table() -> np.ndarray:
    return np.array([e4m3_decode(c) for c in range(256)], dtype=np.float64)


def f32_to_e4m3(x) -> np.ndarray:
    """OCP E4M3FN codes with round-to-nearest-even and saturation to +-448."""
    x = _f32(x)
    out = np.empty(x.shape, dtype=np.uint8)
    _lib().or_f32_to_e4m3(x.ravel(), x.size, out.reshape(-1))
    return out


def e4m3_to_f64(codes) -> np.ndarray:
    return e4m3_table()[np.asarray(codes, dtype=np.uint8)]


def fp8_scale(x) -> tuple:
    """Per-tensor scaling for FP8 (reading of the precision workload):
    amax = max |x| (FP32), inv = 448 / amax and scale = amax / 448, both
    single FP32 divisions; codes = E4M3(x * inv) with the product rounded to
    FP32 first.  Returns (inv, scale) as FP32; amax == 0 gives (1, 1)."""
    x = _f32(x)
    amax = np.float32(np.max(np.abs(x))) if x.size else np.float32(0)
    if amax == 0 or not np.isfinite(amax):
        return np.float32(1.0), np.float32(1.0)
    inv = np.float32(np.float32(448.0) / amax)
    scale = np.float32(amax / np.float32(448.0))
    return inv, scale


def quantize_fp8(x) -> tuple:
    """(codes, scale): codes = E4M3(fl32(x * inv)); dequantised x ~ code * scale."""
    x = _f32(x)
    inv, scale = fp8_scale(x)
    y = (x * inv).astype(np.float32)
    return f32_to_e4m3(y), scale


# --------------------------------------------------------------------------
# Dense victims (Section 4.4.1 uses a GEMM as the shared-memory-sensitive
# victim; decode-phase LLM kernels (Sections 4.2, 4.3) are matrix-vector
# products).  Plain definitions in FP64 on the already-quantised inputs.
# --------------------------------------------------------------------------
def gemm_f64(a, b) -> np.ndarray:
    """C = A @ B^T with A (M x K) and B (N x K), both row-major, in FP64."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return a @ b.T


def gemm_abs_f64(a, b) -> np.ndarray:
    """|A| @ |B|^T: the scale of the rounding-error bound per entry."""
    return np.abs(np.asarray(a, dtype=np.float64)) @ np.abs(np.asarray(b, dtype=np.float64)).T


def gemm_entries_f64(a, b, rows, cols) -> np.ndarray:
    """C[rows[k], cols[k]] of A @ B^T, one dot product per sampled entry."""
    a = np.asarray(a)
    b = np.asarray(b)
    out = np.empty(len(rows), dtype=np.float64)
    for k, (i, j) in enumerate(zip(rows, cols)):
        out[k] = float(np.dot(a[i].astype(np.float64), b[j].astype(np.float64)))
    return out


def gemv_f64(w, x) -> np.ndarray:
    """y = W @ x in FP64, W (N x K) row-major."""
    return np.asarray(w, dtype=np.float64) @ np.asarray(x, dtype=np.float64)


def accumulation_bound(k: int, abs_prod, unit_roundoff: float = 2.0 ** -24):
    """Elementwise bound gamma_k * (|A||B|^T) with gamma_k = k u / (1 - k u)
    (Higham, Accuracy and Stability of Numerical Algorithms, Lemma 3.1), for
    FP32 accumulation of k products that are exact in FP32."""
    ku = k * unit_roundoff
    return (ku / (1.0 - ku)) * np.asarray(abs_prod, dtype=np.float64)


# Characterised behaviour of the FP8 matrix-core instruction (E4M3 x E4M3,
# 32 x 32 x 64, FP32 accumulate) on gfx950, which the instruction set leaves
# unspecified: the 64 products of one output are taken in groups of 8
# consecutive k; within a group every product is aligned to the group's
# largest nominal exponent E (the sum of the two operands' unbiased exponent
# fields, subnormals counted at -6) and cut toward zero to a multiple of
# 2^(E - 13); the group sums and the accumulator input are then added in
# FP32 with round-to-nearest.
FP8_GROUP = 8
FP8_KEEP_BITS = 13


def e4m3_nominal_exponent(codes) -> np.ndarray:
    """Unbiased exponent field of E4M3 codes, subnormals (field 0) at -6."""
    c = np.asarray(codes, dtype=np.uint8)
    return np.maximum((c.astype(np.int32) >> 3) & 15, 1) - 7


def mfma_fp8_error_bound(a_codes, b_codes, scale: float = 1.0, c_abs=0.0) -> np.ndarray:
    """Bound on |computed - exact| for C = scale * A B^T (plus an FP32
    accumulator input of magnitude c_abs) computed with the FP8 instruction
    as characterised above, chained over K in slabs of 64.  a_codes (R x K)
    and b_codes (R x K) hold the rows of A and B of each sampled entry (entry
    r pairs a_codes[r] with b_codes[r]).  Per entry:
      truncation: sum over k of min(|p_k|, 2^(E_g - 13)) over the products
        that are not multiples of their group's quantum (a product loses less
        than one quantum and never more than itself; an E4M3 product is a
        multiple of 2^(e_a + e_b - 6), so one with e_a + e_b - 6 >= E_g - 13
        loses nothing);
      FP32 additions: at most one rounding per group sum plus one for the
        scale: gamma_m(2^-24) (sum |p_k| + c_abs), m = K/8 + 1 (Higham,
        Lemma 3.1 for recursive summation in any order);
    all times |scale|."""
    a = np.asarray(a_codes, dtype=np.uint8)
    b = np.asarray(b_codes, dtype=np.uint8)
    if a.shape != b.shape or a.ndim != 2 or a.shape[1] % FP8_GROUP:
        raise ValueError("a_codes and b_codes must be R x K with K a multiple of 8")
    tab = e4m3_table()
    p = np.abs(tab[a] * tab[b])                              # exact in FP64
    e = (e4m3_nominal_exponent(a) + e4m3_nominal_exponent(b)).astype(np.float64)
    e = np.where(p > 0, e, -np.inf)
    r, k = a.shape
    eg = e.reshape(r, k // FP8_GROUP, FP8_GROUP).max(axis=2)[:, :, None]
    q = np.exp2(eg - FP8_KEEP_BITS)                          # 0 for groups without products
    cut = (e.reshape(r, k // FP8_GROUP, FP8_GROUP) - 6) < (eg - FP8_KEEP_BITS)
    trunc = np.where(cut, np.minimum(p.reshape(r, k // FP8_GROUP, FP8_GROUP), q), 0.0).sum(axis=(1, 2))
    m = k // FP8_GROUP + 1
    u = 2.0 ** -24
    gam = m * u / (1.0 - m * u)
    return abs(scale) * (trunc + gam * (p.sum(axis=1) + np.asarray(c_abs, np.float64)))


def mfma_tile_expected(a_tile, b_tile, iterations: int) -> np.ndarray:
    """Matrix-core stressor: acc <- A B + acc repeated `iterations` times from
    acc = 0, for fixed fragments A (m x k) and B (k x n); exact value
    iterations * (A @ B) in FP64."""
    return float(iterations) * (np.asarray(a_tile, np.float64) @ np.asarray(b_tile, np.float64))


# --------------------------------------------------------------------------
# Slowdown and utilisation (Section 4.1: victim latency colocated versus in
# isolation; Section 2.2: utilisation as a percentage of peak).
# --------------------------------------------------------------------------
def slowdown(t_alone, t_coloc) -> float:
    """median(T_colocated) / median(T_alone)."""
    return float(np.median(np.asarray(t_coloc, np.float64)) /
                 np.median(np.asarray(t_alone, np.float64)))


def bootstrap_slowdown_ci(alone, col, resamples: int = 1000, seed: int = 0) -> tuple:
    """Percentile-bootstrap 95 % interval of median(col) / median(alone), the
    slowdown of Section 4.3 (the paper gives no interval; this is the
    reading the library implements).  Resample r draws len(alone) alone
    times, then len(col) colocated times, with replacement; draw j of
    resample r takes SplitMix64 word r*(na+nc) + j of stream `seed`, modulo
    the sample size.  Quantiles 2.5 % / 97.5 %, linear between order
    statistics."""
    import synth
    a = np.asarray(alone, dtype=np.float64)
    c = np.asarray(col, dtype=np.float64)
    na, nc = a.size, c.size
    k = np.arange(resamples * (na + nc), dtype=np.uint64).reshape(resamples, na + nc)
    w = synth.words_at(seed, k)
    ia = (w[:, :na] % np.uint64(na)).astype(np.int64)
    ic = (w[:, na:] % np.uint64(nc)).astype(np.int64)
    ratios = np.median(c[ic], axis=1) / np.median(a[ia], axis=1)
    return float(np.quantile(ratios, 0.025)), float(np.quantile(ratios, 0.975))


def pct_of_peak(achieved: float, peak: float) -> float:
    return 100.0 * float(achieved) / float(peak)


# --------------------------------------------------------------------------
# Admission rule of the serving loop (reading of Section 5.1: predict each
# kernel's slowdown from its per-resource sensitivity and the co-runners'
# pressure, admit only when every prediction stays within the bound).
# --------------------------------------------------------------------------
SENS_POINTS = (0.0, 0.25, 0.5, 0.75, 1.0)


def curve_at(curve, x: float) -> float:
    """Piecewise-linear slowdown curve measured at intensities SENS_POINTS."""
    x = min(max(float(x), 0.0), 1.0)
    return float(np.interp(x, SENS_POINTS, np.asarray(curve, np.float64)))


def predicted_slowdown(sens, pressure) -> float:
    """sens[r]: the victim's slowdown curve on resource r (five points);
    pressure[r]: summed co-runner pressure on r.  Product over resources of
    max(1, curve_r(pressure_r)) (a conservative combination)."""
    out = 1.0
    for r, curve in enumerate(sens):
        out *= max(1.0, curve_at(curve, pressure[r]))
    return out


READ_MOSTLY_WRITE_FRAC = 1.0 / 6.0


def predicted_slowdown_rw(victim: dict, corunners: list, hbm: int = 0) -> float:
    """The estimator with read/write-aware HBM pricing (reading of Section
    5.1; the HBM axis is split because the same byte rate costs a victim
    more when it includes writes).  victim / corunners: dicts with 'sens'
    (five-point curve per resource), 'press' (load per resource) and
    optionally 'sens_hbm_read' (victim's curve against the read-only HBM
    mix, None or all zeros = absent), 'press_hbm_read' and
    'hbm_write_frac'.  Loads add per resource; HBM load of read-mostly
    co-runners (write share below 1/6) goes on the victim's read-only curve
    when it has one, all other load on its ordinary curve; the factors
    max(1, curve(load)) multiply.  `hbm` is the index of the HBM resource."""
    nres = len(victim["sens"])
    read_curve = victim.get("sens_hbm_read")
    split = read_curve is not None and any(v != 0.0 for v in read_curve)
    load = [0.0] * nres
    load_read = 0.0
    for o in corunners:
        for r in range(nres):
            if r == hbm and split and o.get("hbm_write_frac", 1.0) < READ_MOSTLY_WRITE_FRAC:
                load_read += o.get("press_hbm_read", 0.0)
            else:
                load[r] += o["press"][r]
    out = predicted_slowdown(victim["sens"], load)
    if split:
        out *= max(1.0, curve_at(read_curve, load_read))
    return out


def admit(policy: str, running: list, cand: dict, free_bytes: int, bound: float,
          slots: int, background: dict | None = None) -> bool:
    """running / cand: dicts with 'sens' (per-resource five-point curves),
    'press' (per-resource pressure it exerts), 'bytes' and 'occ' (fraction of wave
    slots).  Policies: 'naive' (memory and slot only), 'usher' (summed
    occupancy below 1, Section 3 Pitfall 1), 'sensitivity' (predicted
    slowdown of every job within `bound`).

    Section 5.1 asks the scheduler to predict each job's slowdown per
    resource but gives no formula; the reading taken here: each curve is
    piecewise linear through its five measured points, co-runner pressures
    on a resource add and clip at 1, the per-resource factors max(1, curve)
    multiply (predicted_slowdown_rw, with read/write-aware HBM pricing), and
    a request is admitted first in first out, without bypass, only if every
    job, itself included, stays within the bound.

    background: the load of a co-runner present all along (Section 4.1 holds
    a stressor's interference constant for a victim's lifetime), a dict with
    'press', 'occ' and the optional read/write fields.  It is one more
    co-runner of every job and adds its occupancy to the 'usher' sum; it is
    not itself bounded, since no request waits on it."""
    if policy not in ("naive", "usher", "sensitivity"):
        raise ValueError(policy)
    if cand["bytes"] > free_bytes or len(running) >= slots:
        return False
    # On an idle device memory and a slot suffice: the occupancy and slowdown
    # rules bound colocation, and a lone request they refused would wait for
    # ever, since nothing running could free up.
    if policy == "naive" or not running:
        return True
    bg = [background] if background is not None else []
    if policy == "usher":
        return sum(j["occ"] for j in running + bg) + cand["occ"] < 1.0
    if policy != "sensitivity":
        raise ValueError(policy)
    group = running + [cand]
    for j in range(len(group)):
        others = group[:j] + group[j + 1:] + bg
        if predicted_slowdown_rw(group[j], others) > bound:
            return False
    return True


class FirstFitArena:
    """Free list of (offset, size) blocks over [0, size), kept sorted by
    offset; requests are rounded up to 256 bytes and take the lowest block
    that fits; a released block merges with free neighbours."""

    def __init__(self, size: int):
        self.free = [(0, int(size))]

    def alloc(self, nbytes: int):
        nbytes = (int(nbytes) + 255) // 256 * 256
        for i, (off, sz) in enumerate(self.free):
            if sz >= nbytes:
                if sz == nbytes:
                    del self.free[i]
                else:
                    self.free[i] = (off + nbytes, sz - nbytes)
                return off
        return None

    def release(self, off: int, nbytes: int):
        nbytes = (int(nbytes) + 255) // 256 * 256
        self.free.append((off, nbytes))
        self.free.sort()
        merged = []
        for o, z in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + z)
            else:
                merged.append((o, z))
        self.free = merged

    def largest_free(self) -> int:
        return max((z for _, z in self.free), default=0)


def simulate_admission(arrivals, jobs, service_s, policy: str, budget: int, bound: float,
                       slots: int, slowed: bool = False, background: dict | None = None):
    """Discrete-event model of the continuous-batching loop (Section 5.1's
    scheduler, in this library's reading): requests arrive at arrivals[i]
    (sorted); at every arrival and completion the queue head is admitted,
    first in first out and without bypass, for as long as admit(...) allows
    it with the jobs running at that instant and the largest free block of a
    first-fit arena of `budget` bytes; an admitted request runs for
    service_s[i] (times its predicted slowdown beside the jobs running when
    it was admitted if `slowed`) and then frees its slot and memory.
    jobs[i]: the request's admit() dict ('sens', 'press', 'occ', 'bytes', and
    the optional read/write-aware fields); background: a load present all
    along, as in admit() (with `slowed` it also slows every request, a lone
    one included).  Returns a list of dicts with
    'admit', 'end', 'slot', 'corunners' (indices running at admission) per
    request, in request order."""
    n = len(arrivals)
    out = [dict(admit=None, end=None, slot=None, corunners=()) for _ in range(n)]
    arena = FirstFitArena(budget)
    running = {}          # request -> (end time, offset, slot)
    free_slots = list(range(slots))
    queue = []
    nxt = 0
    t = 0.0
    done = 0
    while done < n:
        # next event: an arrival or the earliest completion
        t_arr = arrivals[nxt] if nxt < n else math.inf
        t_end = min((e for e, _, _ in running.values()), default=math.inf)
        t = min(t_arr, t_end)
        if t == math.inf:
            raise ValueError("request %d can never be admitted" % queue[0])
        for q in [q for q, (e, _, _) in running.items() if e <= t]:
            e, off, sl = running.pop(q)
            arena.release(off, jobs[q]["bytes"])
            free_slots.append(sl)
            free_slots.sort()
            done += 1
        while nxt < n and arrivals[nxt] <= t:
            queue.append(nxt)
            nxt += 1
        while queue:
            q = queue[0]
            cur = sorted(running)
            ok = admit(policy, [jobs[r] for r in cur], jobs[q], arena.largest_free(), bound, slots,
                       background)
            if not ok:
                break
            off = arena.alloc(jobs[q]["bytes"])
            if off is None:
                break
            queue.pop(0)
            sl = free_slots.pop(0)
            svc = service_s[q]
            co = [jobs[r] for r in cur] + ([background] if background is not None else [])
            if slowed and co:
                svc *= predicted_slowdown_rw(jobs[q], co)
            running[q] = (t + svc, off, sl)
            out[q].update(admit=t, end=t + svc, slot=sl, corunners=tuple(cur))
    return out


def _median(xs):
    return float(np.median(np.asarray(xs, np.float64))) if len(xs) else math.nan
