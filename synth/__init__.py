"""Seeded synthetic inputs shared by the HIP path and the oracle.

This module only draws random numbers; it holds none of the measured
method's arithmetic.  Both the tests and the benchmark build their inputs
here and hand the same bytes to the device library and to the oracle.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), used in its counter form:
word i of stream `seed` is ``mix(seed + (i + 1) * GAMMA)``.  Because every
word is a pure function of (seed, i), any index can be regenerated on its
own, which the sampled checks at full size rely on, and a device fill
(``synth/fill.hip``) reproduces the same words bit for bit.

Derived draws:
  * uniform in [-1, 1):  ((w >> 40) * 2**-23) - 1, exact in FP32;
  * uint32 words:        w >> 32;
  * normal N(0, sigma):  Box-Muller in FP64 from words 2i and 2i+1,
                         scaled by sigma and rounded once to FP32;
  * a random cyclic permutation (one cycle through all n slots): order the
    slots by a key word each, then link each slot to the next in that
    order and the last back to the first.

Seeds: ``16909 + 1000 * config + buffer_id`` (see ``seed_for``).
"""
from __future__ import annotations

import ctypes
import os
import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK64 = (1 << 64) - 1

# Seeded workloads: one id per buffer role.
BUF_B, BUF_C, BUF_A0, BUF_GEMM_A, BUF_GEMM_B, BUF_GEMV_W, BUF_GEMV_X, \
    BUF_CHASE, BUF_CACHE, BUF_LDS, BUF_MFMA, BUF_SERVE, BUF_B2, BUF_C2 = range(14)


def seed_for(config: int, buffer_id: int) -> int:
    """Seed of buffer `buffer_id` in workload configuration `config`."""
    return 16909 + 1000 * int(config) + int(buffer_id)


def _mix(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def words_at(seed: int, idx) -> np.ndarray:
    """SplitMix64 words number `idx` (array of indices) of stream `seed`."""
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = np.uint64(seed & _MASK64) + (idx + np.uint64(1)) * GAMMA
        return _mix(state)


def words(seed: int, n: int, start: int = 0, chunk: int = 1 << 22) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        out[lo:hi] = words_at(seed, np.arange(start + lo, start + hi, dtype=np.uint64))
    return out


def splitmix64_sequence(seed: int, n: int) -> list:
    """The first n outputs of the sequential SplitMix64 generator seeded with
    `seed` (state advanced by GAMMA before each output)."""
    return [int(x) for x in words(seed, n)]


def _uniform_from_words(w: np.ndarray) -> np.ndarray:
    k = (w >> np.uint64(40)).astype(np.float32)          # 24-bit integer, exact
    return k * np.float32(2.0 ** -23) - np.float32(1.0)  # both steps exact


def uniform_f32(seed: int, n: int, start: int = 0) -> np.ndarray:
    """n FP32 values uniform on [-1, 1), indices start..start+n-1."""
    out = np.empty(n, dtype=np.float32)
    chunk = 1 << 22
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        out[lo:hi] = _uniform_from_words(words_at(seed, np.arange(start + lo, start + hi, dtype=np.uint64)))
    return out


def uniform_affine_f32(seed: int, n: int, scale: float, offset: float = 0.0, start: int = 0) -> np.ndarray:
    """uniform_f32(seed, n, start) * scale + offset, each operation rounded
    to FP32 (the device fill does the same two roundings)."""
    u = uniform_f32(seed, n, start)
    t = u * np.float32(scale)
    return (t + np.float32(offset)).astype(np.float32)


def uniform_f32_at(seed: int, idx) -> np.ndarray:
    return _uniform_from_words(words_at(seed, idx))


def u32(seed: int, n: int, start: int = 0) -> np.ndarray:
    return (words(seed, n, start) >> np.uint64(32)).astype(np.uint32)


def u32_at(seed: int, idx) -> np.ndarray:
    return (words_at(seed, idx) >> np.uint64(32)).astype(np.uint32)


def normal_f32(seed: int, n: int, sigma: float = 1.0) -> np.ndarray:
    """n FP32 samples of N(0, sigma**2) (Box-Muller, FP64, one rounding)."""
    out = np.empty(n, dtype=np.float32)
    chunk = 1 << 22
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        i = np.arange(lo, hi, dtype=np.uint64)
        w1 = words_at(seed, np.uint64(2) * i)
        w2 = words_at(seed, np.uint64(2) * i + np.uint64(1))
        u1 = ((w1 >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53   # (0, 1]
        u2 = (w2 >> np.uint64(11)).astype(np.float64) * 2.0 ** -53           # [0, 1)
        z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
        out[lo:hi] = (sigma * z).astype(np.float32)
    return out


def random_cycle_u32(seed: int, n: int) -> np.ndarray:
    """`next` table of a uniformly random cyclic permutation of 0..n-1.

    Slots are ordered by one random key each (ties, which are vanishingly
    rare, fall back to slot order through a stable sort); slot order[k]
    links to order[k+1] and the last slot back to the first, so following
    `next` from any slot visits all n slots before returning."""
    if n <= 0 or n > (1 << 32):
        raise ValueError("cycle length must be in [1, 2**32]")
    keys = words(seed, n)
    order = np.argsort(keys, kind="stable").astype(np.uint32)
    nxt = np.empty(n, dtype=np.uint32)
    nxt[order] = np.roll(order, -1)
    return nxt


# ---------------------------------------------------------------------------
# Device fill (same words, generated on the GPU) for buffers too large to
# draw on the host in reasonable time.  Loaded lazily; needs libsynth.so.
# ---------------------------------------------------------------------------
_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "libsynth.so")
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(path)
        for name in ("synth_fill_uniform_f32", "synth_fill_u32"):
            fn = getattr(lib, name)
            fn.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64,
                           ctypes.c_uint64, ctypes.c_void_p]
            fn.restype = ctypes.c_int
        lib.synth_fill_affine_f32.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64,
                                              ctypes.c_uint64, ctypes.c_float, ctypes.c_float,
                                              ctypes.c_void_p]
        lib.synth_fill_affine_f32.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def device_fill_uniform_f32(ptr: int, n: int, seed: int, start: int = 0, stream: int = 0) -> None:
    rc = _lib().synth_fill_uniform_f32(ptr, n, seed, start, stream)
    if rc != 0:
        raise RuntimeError(f"synth_fill_uniform_f32 failed: hip error {rc}")


def device_fill_u32(ptr: int, n: int, seed: int, start: int = 0, stream: int = 0) -> None:
    rc = _lib().synth_fill_u32(ptr, n, seed, start, stream)
    if rc != 0:
        raise RuntimeError(f"synth_fill_u32 failed: hip error {rc}")


def device_fill_affine_f32(ptr: int, n: int, seed: int, scale: float, offset: float = 0.0,
                           start: int = 0, stream: int = 0) -> None:
    rc = _lib().synth_fill_affine_f32(ptr, n, seed, start, scale, offset, stream)
    if rc != 0:
        raise RuntimeError(f"synth_fill_affine_f32 failed: hip error {rc}")


# --------------------------------------------------------------------------
# Decode-step inputs: which stream fills which tensor, and its value range.
# Weight matrices are uniform on [-1, 1) scaled by 1/sqrt(fan-in); RMS-norm
# gains uniform on [0.75, 1.25); cache entries and the residual-stream
# input uniform on [-1, 1).  Every tensor is drawn in FP32 and rounded to
# BF16 where the model stores BF16.
def decode_tensor_specs(cfg: dict, seed: int) -> list:
    """[(name, layer, stream seed, count, scale, offset)] for the weights
    (layer -1 = after the last layer), then the caches ("k_cache",
    "v_cache", count per cache tensor) and "x_in"."""
    hid, nq, nkv, d, ffn = cfg["hidden"], cfg["n_q"], cfg["n_kv"], cfg["head_dim"], cfg["ffn"]
    L, vocab, batch, ctx = cfg["layers"], cfg["vocab"], cfg["batch"], cfg["max_ctx"]
    inv = lambda k: float(np.float32(1.0) / np.sqrt(np.float32(k)))
    out = []
    for l in range(L):
        b = seed + 16 * l
        out += [("g_attn", l, b + 0, hid, 0.25, 1.0),
                ("w_qkv", l, b + 1, (nq + 2 * nkv) * d * hid, inv(hid), 0.0),
                ("w_o", l, b + 2, hid * nq * d, inv(nq * d), 0.0),
                ("g_mlp", l, b + 3, hid, 0.25, 1.0),
                ("w_gu", l, b + 4, 2 * ffn * hid, inv(hid), 0.0),
                ("w_down", l, b + 5, hid * ffn, inv(ffn), 0.0)]
    b = seed + 16 * L
    out += [("g_final", -1, b + 0, hid, 0.25, 1.0), ("w_lm", -1, b + 1, vocab * hid, inv(hid), 0.0)]
    n_cache = L * batch * nkv * ctx * d
    out += [("k_cache", -1, b + 2, n_cache, 1.0, 0.0), ("v_cache", -1, b + 3, n_cache, 1.0, 0.0),
            ("x_in", -1, b + 4, batch * hid, 1.0, 0.0)]
    return out
