"""Pins of the CPU oracle against facts fixed outside the oracle itself:
published test vectors, closed forms, library routines that compute the
same definition independently, brute force on tiny inputs and numbers the
paper prints.  Each pin is chosen so that a plausible slip in the oracle (a
fused multiply-add where two roundings are meant, a wrong stride or index,
a transposed operand, an off-by-one in a walk) fails it."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------- inputs
def test_splitmix64_published_vector():
    with open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt")) as f:
        want = [int(l) for l in f if l.strip() and not l.startswith("#")]
    assert synth.splitmix64_sequence(1234567, len(want)) == want


def test_uniform_is_exact_grid_and_in_range():
    u = synth.uniform_f32(7, 1 << 16)
    assert u.dtype == np.float32
    assert u.min() >= -1.0 and u.max() < 1.0
    k = (u.astype(np.float64) + 1.0) * 2.0 ** 23
    assert np.all(k == np.round(k))            # multiples of 2**-23
    assert abs(u.mean()) < 4 * math.sqrt(1 / 3 / u.size)
    assert abs(u.var() - 1 / 3) < 0.01
    # counter form: regenerating any index alone gives the same value
    idx = np.array([0, 5, 65535])
    assert np.array_equal(synth.uniform_f32_at(7, idx), u[idx])
    assert np.array_equal(synth.uniform_f32(7, 10, start=100), u[100:110])


def test_normal_moments():
    z = synth.normal_f32(11, 1 << 18, sigma=0.02)
    n = z.size
    assert abs(z.mean()) < 4 * 0.02 / math.sqrt(n)
    assert abs(z.std() / 0.02 - 1.0) < 4 * math.sqrt(0.5 / n)


def test_random_cycle_is_one_cycle():
    for n in (1, 2, 3, 17, 1000):
        nxt = synth.random_cycle_u32(5, n)
        seen, i = set(), 0
        for _ in range(n):
            seen.add(i)
            i = int(nxt[i])
        assert i == 0 and len(seen) == n
        assert oracle.is_single_cycle(nxt)


def test_is_single_cycle_rejects_two_cycles_and_bad_tables():
    assert not oracle.is_single_cycle(np.array([1, 0, 3, 2], np.uint32))   # two 2-cycles
    assert not oracle.is_single_cycle(np.array([0, 1], np.uint32))         # fixed points
    assert not oracle.is_single_cycle(np.array([1, 5, 0], np.uint32))      # out of range
    assert oracle.is_single_cycle(np.array([1, 2, 0], np.uint32))


# ------------------------------------------------------------------ triad
def test_triad_closed_forms():
    n = 4096
    b = synth.uniform_f32(1, n)
    assert np.array_equal(oracle.triad_f32(b, np.zeros(n, np.float32)), b)
    for k in (-20, 0, 7):
        c = np.full(n, 2.0 ** k, np.float32)
        assert np.all(oracle.triad_f32(np.zeros(n, np.float32), c) == np.float32(3 * 2.0 ** k))


def test_triad_has_two_roundings_not_one():
    """a = fl(b + fl(3c)).  In FP64, 3c is exact (26 bits) and so is b + fl(3c)
    for these inputs, so rounding each step once to FP32 gives the definition
    independently of the oracle's own FP32 code path.  A fused version
    (one rounding) must differ somewhere on these inputs."""
    n = 1 << 18
    b, c = synth.uniform_f32(2, n), synth.uniform_f32(3, n)
    t = (3.0 * c.astype(np.float64)).astype(np.float32)
    want = (b.astype(np.float64) + t.astype(np.float64)).astype(np.float32)
    got = oracle.triad_f32(b, c)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    fused = (b.astype(np.float64) + 3.0 * c.astype(np.float64)).astype(np.float32)
    assert np.count_nonzero(fused != want) > 0


def test_triad_sum_identity():
    """|sum a - (sum b + 3 sum c)| <= u * sum(3|c| + |a|), u = 2**-24."""
    n = 1 << 16
    b, c = synth.uniform_f32(4, n), synth.uniform_f32(5, n)
    a = oracle.triad_f32(b, c)
    lhs = abs(oracle.sum_f32_exact(a) - (math.fsum(b.astype(float)) + 3 * math.fsum(c.astype(float))))
    assert lhs <= 2.0 ** -24 * float(np.sum(3 * np.abs(c.astype(np.float64)) + np.abs(a)))


def test_triad_threads_matches_definition():
    """The threaded form used for the host baseline computes the same
    elements as the FP64 two-rounding definition, for thread counts that do
    and do not divide n (ragged shares, more threads than elements)."""
    for n in (0, 1, 7, 1000003):
        b, c = synth.uniform_f32(6, n), synth.uniform_f32(7, n)
        t = (3.0 * c.astype(np.float64)).astype(np.float32)
        want = (b.astype(np.float64) + t.astype(np.float64)).astype(np.float32)
        for threads in (1, 3, 8, 13):
            got, ran = oracle.triad_f32_threads(b, c, threads)
            assert 1 <= ran <= threads
            assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), (n, threads)


# --------------------------------------------------------------- checksums
def test_bitsum_brute_force_and_wrap():
    x = np.array([1.0, -2.5, 0.0], np.float32)
    assert oracle.bitsum_u32(x) == sum(int(v) for v in x.view(np.uint32)) % 2 ** 64
    w = np.full(5, 0xFFFFFFFF, np.uint32)
    assert oracle.bitsum_u32(w) == 5 * 0xFFFFFFFF
    big = np.full(1 << 20, 0xFFFFFFFF, np.uint32)
    assert oracle.bitsum_u32(big) == ((1 << 20) * 0xFFFFFFFF) % 2 ** 64


def test_exact_sum_against_fsum_and_cancellation():
    x = synth.uniform_f32(9, 100000) * np.float32(1e3)
    assert oracle.sum_f32_exact(x) == math.fsum(x.astype(float))
    y = np.array([3e38, 1.0, -3e38, 2.0 ** -149, -1.0], np.float32)
    assert oracle.sum_f32_exact(y) == 2.0 ** -149
    z = np.array([-1.5, -2.25], np.float32)
    assert oracle.sum_f32_exact(z) == -3.75
    assert math.isnan(oracle.sum_f32_exact(np.array([1.0, np.inf], np.float32)))


def test_rel_err_sum_switches_to_normwise_on_cancellation():
    x = np.array([1.0, -1.0, 1e-6], np.float32)
    # sum ~ 1e-6 << 1e-3 * sum|x| ~ 2e-3 -> normwise, denominator ~ 2
    assert oracle.rel_err_sum(0.0, x) == pytest.approx(float(np.float32(1e-6)) / 2.000001, rel=1e-6)


def test_cache_sums_closed_form():
    for n in (1, 7, 4096, 1 << 20):
        w = np.arange(n, dtype=np.uint32)
        assert oracle.region_sum_u32(w) == (n * (n - 1) // 2) % 2 ** 32
    w = np.arange(1 << 20, dtype=np.uint32)
    exp = oracle.cache_wg_expected(w, [0, 1, 3, 1000003])
    s = ((1 << 20) * ((1 << 20) - 1) // 2) % 2 ** 32
    assert list(exp) == [0, s, (3 * s) % 2 ** 32, (1000003 * s) % 2 ** 32]


def test_hbm_mix_closed_forms():
    # read-only: b holds the words 0..n-1, c a constant K -> passes * (n(n-1)/2 + nK) mod 2^32
    for n, k, p in ((1, 5, 1), (1000, 0xFFFFFFFF, 3), ((1 << 20) + 77, 0x9E3779B1, 7)):
        b = np.arange(n, dtype=np.uint32).view(np.float32)
        c = np.full(n, k, np.uint32).view(np.float32)
        assert oracle.hbm_read_checksum(b, c, p) == (p * (n * (n - 1) // 2 + n * k)) % 2 ** 32
    # copy keeps every bit, signalling-NaN payloads included
    w = np.array([0x7F800001, 0xFFC00123, 0x80000000, 0x3F800000], np.uint32)
    assert np.array_equal(oracle.hbm_copy(w.view(np.float32)), w)
    # write-only: an odd multiplier is a bijection mod 2^32, indices wrap at 2^32,
    # and the words sum to K n(n-1)/2 mod 2^32
    k = oracle.WRITE_MULTIPLIER
    assert k % 2 == 1
    pat = oracle.hbm_write_pattern(1 << 16)
    assert pat[0] == 0 and pat[1] == k and len(np.unique(pat)) == 1 << 16
    n = (1 << 20) + 13
    assert oracle.region_sum_u32(oracle.hbm_write_pattern(n)) == (k * (n * (n - 1) // 2)) % 2 ** 32
    assert np.array_equal(oracle.hbm_write_pattern(5, first=(1 << 32) + 9), oracle.hbm_write_pattern(5, first=9))
    assert [oracle.hbm_bytes_per_element(m) for m in ("triad", "read", "copy", "write")] == [12, 8, 8, 4]


def test_lds_pass_visits_every_vector_once_per_lane():
    """Each lane walks all nvec vectors once per pass, for any stride, so a
    wave's pass sum is 64 * sum(window); brute force on a tiny window also
    pins the stride and index arithmetic."""
    w = synth.u32(21, 8192)
    total = int(w.astype(np.uint64).sum()) % 2 ** 32
    for vw in (1, 2, 4):
        for stride in (1, 2, 3, 32, 64):
            assert oracle.lds_wave_pass_sum(w, vw, stride) == (64 * total) % 2 ** 32
    tiny = np.arange(12, dtype=np.uint32) * np.uint32(7) + np.uint32(1)
    for vw, stride in ((1, 5), (2, 4), (4, 3)):
        nvec = 12 // vw
        s = 0
        for lane in range(64):
            for k in range(nvec):
                v = (lane * stride + k) % nvec
                s += int(tiny[v * vw:(v + 1) * vw].sum())
        assert oracle.lds_wave_pass_sum(tiny, vw, stride) == s % 2 ** 32


# ------------------------------------------------------------- VALU chain
def test_fma_chain_closed_forms():
    z = np.zeros(3, np.float32)
    assert np.all(oracle.fma_chain_f32(z, 1.0, 1.0, 1000) == 1000.0)
    out = oracle.fma_chain_f32(z, 0.5, 1.0, 10)
    assert np.all(out == np.float32(2 - 2.0 ** -9))
    assert np.all(oracle.fma_chain_f32(z, 0.5, 1.0, 30) == 2.0)


def test_fma_chain_rounds_once():
    """x*a = 1 + 2**-11 + 2**-24 exactly; fma(x, a, -1) keeps the 2**-24
    term, whereas rounding the product first would lose it."""
    x = np.array([1 + 2.0 ** -12], np.float32)
    out = oracle.fma_chain_f32(x, 1 + 2.0 ** -12, -1.0, 1)
    assert out[0] == np.float32(2.0 ** -11 + 2.0 ** -24)


def test_valu_start_values_and_fixed_point():
    th = np.array([0, 1, 1023, 1024, 5000])
    x0 = oracle.valu_start_values(th, 4)
    assert x0[0, 0] == np.float32(2.0 ** -10) and x0[3, 0] == x0[0, 0]
    assert x0[2, 3] == np.float32((1023 + 3 + 1) * 2.0 ** -10)
    # x_{k} - 1 = a^k (x0 - 1) with a = 1 - 2**-12, b = 2**-12: converges to 1
    out = oracle.valu_outputs(th, 4, 1 - 2.0 ** -12, 2.0 ** -12, 4096)
    exact = 1 + (1 - 2.0 ** -12) ** 4096 * (x0.astype(np.float64) - 1)
    assert np.max(np.abs(out - exact)) < 4096 * 2.0 ** -23


def test_dmul_chain_closed_forms_and_rounding():
    x0 = np.array([0.75, 1.0, 3.0], np.float64)
    assert np.array_equal(oracle.dmul_chain_f64(x0, 2.0, 100), x0 * 2.0 ** 100)
    assert np.array_equal(oracle.dmul_chain_f64(x0, 0.5, 50), x0 * 2.0 ** -50)
    # one correctly rounded binary64 multiply per step, checked with exact
    # rational arithmetic on a product that needs rounding
    a = 1 + 2.0 ** -30
    x = 1 + 2.0 ** -29
    got = oracle.dmul_chain_f64(np.array([x]), a, 1)[0]
    exact = Fraction(x) * Fraction(a)          # 1 + 3*2^-30 + 2^-59: needs rounding
    assert Fraction(got) != exact and abs(Fraction(got) - exact) <= Fraction(2.0 ** -53)
    assert got == x * a
    out = oracle.valu64_outputs(np.array([0, 1023, 1024]), 2, 0.5, 3)
    assert out[0, 0] == 2.0 ** -10 / 8 and out[2, 1] == out[0, 1] == 2 * 2.0 ** -10 / 8


# ----------------------------------------------------------- pointer chase
def test_chase_brute_force_and_full_cycle():
    n = 1 << 12
    nxt = synth.random_cycle_u32(13, n)
    starts = np.array([0, 1, 4095, 77], np.uint64)
    for hops in (0, 1, 5, 1000):
        want = []
        for s in starts:
            i = int(s)
            for _ in range(hops):
                i = int(nxt[i])
            want.append(i)
        assert list(oracle.chase_u32(nxt, starts, hops)) == want
    assert np.array_equal(oracle.chase_u32(nxt, starts, n), starts.astype(np.uint32))
    assert not np.array_equal(oracle.chase_u32(nxt, starts, n - 1), starts.astype(np.uint32))


# ----------------------------------------------------------------- BF16
def test_bf16_ties_overflow_nan():
    f = lambda bits: np.array([bits], np.uint32).view(np.float32)
    # halfway between 1.0 (0x3F80) and 1 + 2**-7 (0x3F81): even code wins
    assert oracle.f32_to_bf16(f(0x3F808000))[0] == 0x3F80
    # halfway between 0x3F81 and 0x3F82: even code wins (0x3F82)
    assert oracle.f32_to_bf16(f(0x3F818000))[0] == 0x3F82
    assert oracle.f32_to_bf16(f(0x3F808001))[0] == 0x3F81
    assert oracle.f32_to_bf16(f(0x3F807FFF))[0] == 0x3F80
    assert oracle.f32_to_bf16(f(0xBF808001))[0] == 0xBF81
    # largest finite FP32 rounds to +inf in BF16 (beyond the overflow midpoint)
    assert oracle.f32_to_bf16(f(0x7F7FFFFF))[0] == 0x7F80
    assert oracle.f32_to_bf16(f(0x7F7F7FFF))[0] == 0x7F7F
    assert oracle.f32_to_bf16(np.array([np.inf, -np.inf], np.float32)).tolist() == [0x7F80, 0xFF80]
    assert oracle.f32_to_bf16(np.array([np.nan], np.float32))[0] & 0x7FC0 == 0x7FC0


def test_bf16_nearest_by_brute_force():
    x = synth.normal_f32(17, 5000)
    codes = oracle.f32_to_bf16(x)
    for v, c in zip(x[:500], codes[:500]):
        t = int(np.array([v], np.float32).view(np.uint32)[0]) >> 16
        cands = [t, t + 1]
        vals = [Fraction(float(oracle.bf16_to_f64(np.array([cc], np.uint16))[0])) for cc in cands]
        err = [abs(Fraction(float(v)) - q) for q in vals]
        best = cands[0] if err[0] < err[1] else cands[1] if err[1] < err[0] else \
            (cands[0] if cands[0] % 2 == 0 else cands[1])
        assert c == best


# ------------------------------------------------------------------- FP8
def test_e4m3_named_values():
    with open(os.path.join(GOLDEN, "e4m3_points.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    for code, val in rows:
        got = oracle.e4m3_decode(int(code, 16))
        assert got == float(val) and math.copysign(1, got) == math.copysign(1, float(val))
    assert math.isnan(oracle.e4m3_decode(0x7F)) and math.isnan(oracle.e4m3_decode(0xFF))
    t = oracle.e4m3_table()
    finite = t[np.isfinite(t)]
    assert finite.size == 254 and np.max(finite) == 448.0


def test_e4m3_round_trip_ties_and_saturation():
    t = oracle.e4m3_table()
    codes = np.array([c for c in range(256) if np.isfinite(t[c])], np.uint8)
    vals = t[codes].astype(np.float32)
    back = oracle.f32_to_e4m3(vals)
    # +0 and -0 keep their own codes; every finite code round-trips
    assert np.array_equal(back, codes)
    # midpoint between 1.0 (0x38, even) and 1.125 (0x39) -> 0x38;
    # midpoint between 1.125 and 1.25 (0x3A, even) -> 0x3A
    assert oracle.f32_to_e4m3(np.array([1.0625, 1.1875], np.float32)).tolist() == [0x38, 0x3A]
    # saturation: beyond 448, infinities -> +-448; NaN -> NaN code
    assert oracle.f32_to_e4m3(np.array([464.0, 1e9, np.inf, -np.inf], np.float32)).tolist() == \
        [0x7E, 0x7E, 0x7E, 0xFE]
    assert oracle.f32_to_e4m3(np.array([np.nan], np.float32))[0] & 0x7F == 0x7F
    # below half the smallest subnormal -> zero; at exactly half -> zero (even)
    assert oracle.f32_to_e4m3(np.array([2.0 ** -11, 2.0 ** -10, 2.0 ** -10 * 1.01], np.float32)).tolist() \
        == [0, 0, 1]


def test_fp8_scale_and_quantize():
    x = np.array([0.5, -2.0, 1.0], np.float32)
    inv, scale = oracle.fp8_scale(x)
    assert inv == np.float32(224.0) and scale == np.float32(2.0 / 448.0)
    codes, s = oracle.quantize_fp8(x)
    assert oracle.e4m3_decode(codes[1]) == -448.0
    assert np.allclose(oracle.e4m3_to_f64(codes) * s, x, rtol=2 ** -4)
    assert oracle.fp8_scale(np.zeros(4, np.float32)) == (1.0, 1.0)


# ---------------------------------------------------------------- GEMM/V
def test_gemm_oracle_against_loops_and_identity():
    rng_a = synth.normal_f32(31, 5 * 7).reshape(5, 7)
    rng_b = synth.normal_f32(32, 3 * 7).reshape(3, 7)
    c = oracle.gemm_f64(rng_a, rng_b)
    for i in range(5):
        for j in range(3):
            s = math.fsum(float(rng_a[i, k]) * float(rng_b[j, k]) for k in range(7))
            assert abs(c[i, j] - s) < 1e-12
    eye = np.eye(7, dtype=np.float32)
    assert np.array_equal(oracle.gemm_f64(rng_a, eye), rng_a.astype(np.float64))
    # B^T convention: a non-symmetric B must not be used untransposed
    b = np.arange(49, dtype=np.float32).reshape(7, 7)
    assert np.array_equal(oracle.gemm_f64(eye, b), b.T.astype(np.float64))
    ent = oracle.gemm_entries_f64(rng_a, rng_b, [0, 4, 2], [2, 0, 1])
    assert np.allclose(ent, [c[0, 2], c[4, 0], c[2, 1]], rtol=0, atol=1e-12)


def test_gemv_row_sums():
    w = synth.normal_f32(33, 6 * 9, sigma=0.02).reshape(6, 9)
    y = oracle.gemv_f64(w, np.ones(9, np.float32))
    for i in range(6):
        assert abs(y[i] - math.fsum(float(v) for v in w[i])) < 1e-15


def _toy_rne(x, bits):
    """x (Fraction) rounded to nearest, ties to even, at `bits` significand bits."""
    if x == 0:
        return x
    a = abs(x)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    ulp = Fraction(2) ** (e - bits + 1)
    q, r = divmod(a, ulp)
    q = int(q)
    if r > ulp / 2 or (r == ulp / 2 and q % 2):
        q += 1
    return (1 if x > 0 else -1) * q * ulp


def test_accumulation_bound_against_brute_force_worst_case():
    """Recursive summation in a toy binary format with 3-bit significands
    (unit roundoff 2^-3), every sequence of 2 and 3 terms from 40 values,
    exact rational arithmetic: the error never exceeds the bound for n - 1
    roundings, and comes within 0.78 (n = 2) and 0.6 (n = 3) of it, so a
    bound with half the unit, or one rounding fewer, would fail."""
    import itertools
    bits = 3
    u = 2.0 ** -bits
    vals = sorted({s * Fraction(m, 2 ** (bits - 1)) * Fraction(2) ** e
                   for m in range(2 ** (bits - 1), 2 ** bits) for e in range(-2, 3) for s in (1, -1)})
    for n, tight in ((2, 0.77), (3, 0.59)):
        worst = 0.0
        for seq in itertools.product(vals, repeat=n):
            acc = seq[0]
            for x in seq[1:]:
                acc = _toy_rne(acc + x, bits)
            err = float(abs(acc - sum(seq)))
            bound = float(oracle.accumulation_bound(n - 1, float(sum(abs(x) for x in seq)), u))
            assert err <= bound, seq
            worst = max(worst, err / bound)
        assert worst >= tight
        # with one rounding fewer the same worst case breaks the bound (n = 3)
        if n == 3:
            assert worst * float(oracle.accumulation_bound(2, 1.0, u)) > float(oracle.accumulation_bound(1, 1.0, u))


def test_accumulation_bound_and_mfma_closed_form():
    b = oracle.accumulation_bound(4096, np.ones((2, 2)))
    assert np.allclose(b, 4096 * 2.0 ** -24 / (1 - 4096 * 2.0 ** -24))
    a = np.ones((32, 16))
    bb = np.ones((16, 32))
    assert np.all(oracle.mfma_tile_expected(a, bb, 1000) == 16000.0)
    a2 = np.arange(6, dtype=float).reshape(2, 3)
    b2 = np.arange(6, dtype=float).reshape(3, 2)
    assert np.array_equal(oracle.mfma_tile_expected(a2, b2, 2), 2 * np.array([[10, 13], [28, 40]]))


# ------------------------------------------------------ paper's own numbers
def test_slowdown_definition_against_paper_table1():
    with open(os.path.join(GOLDEN, "paper_numbers.json")) as f:
        p = json.load(f)
    t = p["table1_membw"]
    s = oracle.slowdown([t["p90_tbt_ms"][0]], [t["p90_tbt_ms"][-1]])
    assert round(s, 2) == t["max_slowdown_stated"]
    fv = p["full_vs_partition"]
    assert round(oracle.slowdown([fv["full_ms"]], [fv["partition_ms"]]), 2) == fv["slowdown_stated"]
    bs = p["block_scheduler"]
    assert oracle.slowdown([bs["alone_ms"]] * 3, [bs["coloc_ms"]] * 3) > 2.0
    # median, not mean: one outlier does not move it
    assert oracle.slowdown([1.0, 1.0, 1.0], [1.0, 1.0, 100.0]) == 1.0
    occ = p["occupancy"]
    assert oracle.pct_of_peak(occ["warps_per_block"], occ["max_warps_per_sm"]) == occ["occupancy_pct"]


# ------------------------------------------------------------- admission
def _job(sens1, press, nbytes=1, occ=0.1):
    curves = [[1.0 + (s - 1.0) * t for t in oracle.SENS_POINTS] for s in sens1]
    return {"sens": curves, "press": press, "bytes": nbytes, "occ": occ}


def test_bootstrap_ci_closed_forms():
    # constant samples: every resample gives the same ratio
    assert oracle.bootstrap_slowdown_ci([2.0] * 5, [3.0] * 4, 200, 1) == (1.5, 1.5)
    assert oracle.bootstrap_slowdown_ci([8.0], [2.0], 50, 3) == (0.25, 0.25)
    # alone {1, 2, 10}, colocated {4}: the median of three draws is 1 or 10
    # with probability 7/27 each, else 2, so ratios are 4, 2 or 0.4 and the
    # 2.5 % / 97.5 % quantiles of 1000 resamples sit on 0.4 and 4 (a mean
    # instead of the median, or swapped samples, would move them)
    lo, hi = oracle.bootstrap_slowdown_ci([1.0, 2.0, 10.0], [4.0], 1000, 7)
    assert (lo, hi) == (0.4, 4.0)
    # draws use the counter-form generator: a different seed, same law
    assert oracle.bootstrap_slowdown_ci([1.0, 2.0, 10.0], [4.0], 1000, 8) == (0.4, 4.0)


def test_admission_rules():
    quiet = _job([1.0, 1.0], [0.0, 0.0])
    hog = _job([1.0, 1.0], [1.0, 0.0], occ=0.6)
    fragile = _job([3.0, 1.0], [0.0, 0.0], occ=0.6)
    # memory and slots bind every policy
    for pol in ("naive", "usher", "sensitivity"):
        assert not oracle.admit(pol, [], _job([1, 1], [0, 0], nbytes=10), 5, 1.5, 4)
        assert not oracle.admit(pol, [quiet] * 4, quiet, 10, 1.5, 4)
    assert oracle.admit("naive", [hog], fragile, 10, 1.5, 4)
    assert not oracle.admit("usher", [hog], fragile, 10, 1.5, 4)     # occupancy 1.2
    assert not oracle.admit("sensitivity", [hog], fragile, 10, 1.5, 4)  # predicts 3x
    assert oracle.admit("sensitivity", [hog], fragile, 10, 3.0, 4)
    assert oracle.admit("sensitivity", [quiet], fragile, 10, 1.5, 4)
    # unbounded: sensitivity == naive
    assert oracle.admit("sensitivity", [hog, hog], fragile, 10, math.inf, 4)
    # piecewise-linear interpolation between the measured points
    assert oracle.predicted_slowdown([[1.0, 1.5, 2.0, 2.5, 3.0]], [0.5]) == 2.0
    assert oracle.predicted_slowdown([[1.0, 1.0, 1.0, 2.0, 4.0]], [0.875]) == 3.0
    # pressure is clipped to [0, 1]; slowdowns below 1 count as 1; product over resources
    assert oracle.predicted_slowdown([[1.0, 1.0, 1.0, 1.0, 2.0]], [5.0]) == 2.0
    assert oracle.predicted_slowdown([[0.9] * 5, [2.0] * 5], [0.3, 0.3]) == 2.0
    assert oracle.predicted_slowdown([[1.5] * 5, [2.0] * 5], [0.3, 0.3]) == 3.0


# ----------------------------------------- characterised FP8 matrix core
def _fp8_instruction_model(a_codes, b_codes, c0=0.0):
    """The characterised accumulation, written out with exact rationals:
    groups of 8 consecutive products, each cut toward zero to a multiple of
    2^(E - 13) (E the group's largest sum of exponent fields), group sums
    added one after another to the FP32 accumulator with round-to-nearest."""
    tab = oracle.e4m3_table()
    acc = Fraction(float(np.float32(c0)))
    for g0 in range(0, len(a_codes), 8):
        prods, exps = [], []
        for k in range(g0, g0 + 8):
            p = Fraction(float(tab[a_codes[k]])) * Fraction(float(tab[b_codes[k]]))
            prods.append(p)
            if p != 0:
                exps.append(int(oracle.e4m3_nominal_exponent(a_codes[k]) + oracle.e4m3_nominal_exponent(b_codes[k])))
        if not exps:
            continue
        q = Fraction(2) ** (max(exps) - 13)
        gsum = sum((1 if p > 0 else -1) * (abs(p) // q) * q for p in prods)
        acc = _toy_rne(acc + gsum, 24)
    return acc


def _e4m3_code(v):
    tab = oracle.e4m3_table()
    return int(np.flatnonzero(tab == v)[0])


def test_fp8_bound_hand_case():
    # one group: products 256 (1 x 256) and 2^-6 (1 x 2^-6); E = 8, quantum
    # 2^-5; 256 is a multiple of it (granularity 2^(8-6)) and keeps all its
    # bits, 2^-6 is below it and may be lost whole
    a = np.zeros((1, 8), np.uint8)
    b = np.zeros((1, 8), np.uint8)
    a[0, 0] = a[0, 1] = _e4m3_code(1.0)
    b[0, 0], b[0, 1] = _e4m3_code(256.0), _e4m3_code(2.0 ** -6)
    got = oracle.mfma_fp8_error_bound(a, b)[0]
    u = 2.0 ** -24
    want = 2.0 ** -6 + 2 * u / (1 - 2 * u) * (256 + 2.0 ** -6)
    assert got == pytest.approx(want, rel=1e-15)
    # scale and the accumulator input enter linearly
    assert oracle.mfma_fp8_error_bound(a, b, scale=-2.0, c_abs=8.0)[0] == pytest.approx(
        2 * (2.0 ** -6 + 2 * u / (1 - 2 * u) * (256 + 2.0 ** -6 + 8.0)), rel=1e-15)
    # 1 x 1 and 1 x 2^-6: E = 0, quantum 2^-13; 2^-6 has granularity
    # 2^(-6-6) = 2^-12, a multiple of the quantum, and loses nothing
    b[0, 0] = _e4m3_code(1.0)
    assert oracle.mfma_fp8_error_bound(a, b)[0] == pytest.approx(2 * u / (1 - 2 * u) * (1 + 2.0 ** -6),
                                                                 rel=1e-15)
    # a group that spans less than 8 bits of exponent loses nothing to truncation
    a[0, :] = _e4m3_code(1.5)
    b[0, :] = _e4m3_code(0.75)
    p = 8 * 1.125
    assert oracle.mfma_fp8_error_bound(a, b)[0] == pytest.approx(2 * u / (1 - 2 * u) * p, rel=1e-15)


def test_fp8_bound_dominates_the_model_and_is_tight():
    """On seeded random codes and on adversarial tiles (one large product,
    small ones just below the group's quantum, with and without the large
    pair cancelling), the bound covers the model's error everywhere, and the
    adversarial tiles reach at least half of it: a bound with 14 kept bits
    (half the quantum) would fail there."""
    rng = np.random.default_rng(16909)
    fin = np.flatnonzero(np.isfinite(oracle.e4m3_table()))
    tab = oracle.e4m3_table()
    worst = 0.0
    cases = []
    for _ in range(150):
        cases.append((rng.choice(fin, 64).astype(np.uint8), rng.choice(fin, 64).astype(np.uint8), rng.normal() * 10))
    one, big, small = _e4m3_code(1.0), _e4m3_code(256.0), _e4m3_code(2.0 ** -5.0) if np.any(tab == 2.0 ** -5) else None
    for cancel in (False, True):
        a = np.full(64, one, np.uint8)
        b = np.full(64, _e4m3_code(2.0 ** -6), np.uint8)
        b[0] = big                                  # 2^8 against 2^-6 products: gap 14 bits
        if cancel:
            a[1], b[1] = _e4m3_code(-1.0), big
        cases.append((a, b, 0.0))
    for a, b, c0 in cases:
        exact = sum(Fraction(float(tab[x])) * Fraction(float(tab[y])) for x, y in zip(a, b)) + Fraction(float(np.float32(c0)))
        err = abs(float(_fp8_instruction_model(a, b, c0) - exact))
        bound = oracle.mfma_fp8_error_bound(a[None, :], b[None, :], 1.0, abs(float(np.float32(c0))))[0]
        assert err <= bound
        worst = max(worst, err / bound)
    assert worst >= 0.5


# ------------------------------------------- estimator with the HBM split
def _prof(hbm_curve, read_curve=None, press_hbm=0.0, press_read=0.0, wfrac=1.0, extra=None):
    sens = [list(hbm_curve), [1.0] * 5]
    press = [press_hbm, 0.0 if extra is None else extra]
    p = {"sens": sens, "press": press, "hbm_write_frac": wfrac, "press_hbm_read": press_read,
         "bytes": 1, "occ": 0.1}
    if read_curve is not None:
        p["sens_hbm_read"] = list(read_curve)
    return p


def test_read_write_aware_estimator_hand_cases():
    triad = [1.0, 2.0, 3.0, 4.0, 5.0]
    reads = [1.0, 1.2, 1.4, 1.6, 1.8]
    victim = _prof(triad, reads)
    plain_victim = _prof(triad)
    reader = _prof(triad, press_hbm=0.9, press_read=0.5, wfrac=0.0)      # read-mostly co-runner
    writer = _prof(triad, press_hbm=0.5, press_read=0.9, wfrac=1 / 3)    # triad-like co-runner
    # a read-mostly co-runner is priced on the read curve at its read-mix load
    assert oracle.predicted_slowdown_rw(victim, [reader]) == pytest.approx(1.4)
    # without a read curve the victim prices it on the ordinary curve at its HBM load
    assert oracle.predicted_slowdown_rw(plain_victim, [reader]) == pytest.approx(4.6)
    # a co-runner that writes is priced on the ordinary curve
    assert oracle.predicted_slowdown_rw(victim, [writer]) == pytest.approx(3.0)
    # both: the two HBM factors multiply
    assert oracle.predicted_slowdown_rw(victim, [reader, writer]) == pytest.approx(1.4 * 3.0)
    # a write share of exactly 1/6 is not read-mostly
    edge = _prof(triad, press_hbm=0.25, press_read=0.75, wfrac=1 / 6)
    assert oracle.predicted_slowdown_rw(victim, [edge]) == pytest.approx(2.0)
    # loads add and clip at 1; other resources multiply in
    two_readers = oracle.predicted_slowdown_rw(victim, [reader, reader])
    assert two_readers == pytest.approx(1.8)
    other = _prof(triad, press_hbm=0.0, wfrac=0.0, extra=0.5)
    v2 = dict(victim, sens=[triad, [1.0, 1.0, 2.0, 3.0, 4.0]])
    assert oracle.predicted_slowdown_rw(v2, [other]) == pytest.approx(2.0)
    # no co-runner: 1; the estimator without read curves is the plain product rule
    assert oracle.predicted_slowdown_rw(victim, []) == 1.0
    assert oracle.predicted_slowdown_rw(plain_victim, [writer]) == oracle.predicted_slowdown(
        plain_victim["sens"], [0.5, 0.0])


def test_admission_lets_a_lone_request_in():
    """On an idle device a request needs only memory and a slot: neither the
    occupancy rule nor the slowdown bound can refuse it (nothing would ever
    free up); beside a co-runner they apply as before."""
    greedy = _job([5.0, 1.0], [1.0, 0.0], occ=1.0)
    for pol in ("usher", "sensitivity"):
        assert oracle.admit(pol, [], greedy, 10, 1.01, 4)
        assert not oracle.admit(pol, [greedy], greedy, 10, 1.01, 4)
        assert not oracle.admit(pol, [], _job([1, 1], [0, 0], nbytes=20), 10, 1.01, 4)
    with pytest.raises(ValueError):
        oracle.admit("fifo", [], greedy, 10, 1.5, 4)



def test_admission_with_a_background_load():
    """A load present all along (a stressor held for the whole run) is one
    more co-runner of every job and adds its occupancy to the occupancy sum,
    but is not bounded itself.  Hand cases with dyadic loads on linear
    curves (slowdown 1 + x on the first resource), and the identity that
    ties it to the pinned rule: admitting beside a background X is admitting
    beside X as a running job, less X's own bound."""
    run = _job([2.0, 1.0], [0.25, 0.0], occ=0.25)
    cand = _job([2.0, 1.0], [0.125, 0.0], occ=0.25)
    bg = {"press": [0.5, 0.0], "occ": 0.5}
    # cand beside run and bg: 1 + 0.25 + 0.5 = 1.75; run beside cand and bg: 1.625
    assert oracle.predicted_slowdown_rw(cand, [run, bg]) == 1.75
    assert oracle.predicted_slowdown_rw(run, [cand, bg]) == 1.625
    assert oracle.admit("sensitivity", [run], cand, 10, 1.7, 4)               # 1.25 and 1.125
    assert not oracle.admit("sensitivity", [run], cand, 10, 1.7, 4, background=bg)
    assert oracle.admit("sensitivity", [run], cand, 10, 1.75, 4, background=bg)
    # occupancy: 0.25 + 0.25 + 0.5 = 1 is not below 1; 0.375 leaves room
    assert oracle.admit("usher", [run], cand, 10, 1.5, 4)
    assert not oracle.admit("usher", [run], cand, 10, 1.5, 4, background=bg)
    assert oracle.admit("usher", [run], cand, 10, 1.5, 4, background=dict(bg, occ=0.375))
    # the background's own slowdown is never bounded: a background that a
    # running job would slow 100x changes nothing
    assert oracle.admit("sensitivity", [run], cand, 10, 1.75, 4,
                        background=dict(bg, sens=[[100.0] * 5, [100.0] * 5]))
    # memory, slots and the idle-device rule are untouched
    assert oracle.admit("sensitivity", [], cand, 10, 1.01, 4, background={"press": [1.0, 1.0], "occ": 1.0})
    assert not oracle.admit("naive", [], _job([1, 1], [0, 0], nbytes=20), 10, 1.5, 4, background=bg)
    assert not oracle.admit("naive", [run] * 4, cand, 10, 1.5, 4, background=bg)
    assert oracle.admit("naive", [run], cand, 10, 1.0, 4, background={"press": [1.0, 1.0], "occ": 2.0})
    rng = np.random.default_rng(21)
    for _ in range(400):
        kinds = [_job([1.0 + 3.0 * rng.random(), 1.0 + rng.random()], [rng.random(), rng.random()],
                      occ=0.5 * rng.random()) for _ in range(4)]
        running = [kinds[int(i)] for i in rng.integers(0, 4, int(rng.integers(1, 4)))]
        cand = kinds[int(rng.integers(0, 4))]
        x = kinds[int(rng.integers(0, 4))]
        bound = 1.0 + 3.0 * rng.random()
        zero = {"press": [0.0, 0.0], "occ": 0.0}
        for pol in ("naive", "usher", "sensitivity"):
            plain = oracle.admit(pol, running, cand, 10, bound, 8)
            assert oracle.admit(pol, running, cand, 10, bound, 8, background=zero) == plain
            beside_x = oracle.admit(pol, running + [x], cand, 10, bound, 8)
            with_bg = oracle.admit(pol, running, cand, 10, bound, 8, background=x)
            if pol == "sensitivity":
                own = oracle.predicted_slowdown_rw(x, running + [cand])
                assert beside_x == (with_bg and own <= bound)
            else:
                assert beside_x == with_bg


def test_simulator_with_a_background_load():
    """A background that alone predicts more than the bound for every
    request serialises sensitivity admission (a lone request is still
    admitted) and, with slowed service, stretches a lone request by its
    predicted slowdown beside the background alone."""
    frag = _job([3.0, 1.0], [0.0, 0.0], nbytes=1, occ=0.25)
    bg = {"press": [0.5, 0.0], "occ": 0.5}           # 1 + 2 * 0.5 = 2x for each request
    out = oracle.simulate_admission([0.0, 0.5], [frag, frag], [2.0, 2.0], "sensitivity", 1024, 1.5, 4)
    assert [(o["admit"], o["end"]) for o in out] == [(0.0, 2.0), (0.5, 2.5)]   # zero press: together
    out = oracle.simulate_admission([0.0, 0.5], [frag, frag], [2.0, 2.0], "sensitivity", 1024, 1.5, 4,
                                    background=bg)
    assert [(o["admit"], o["end"]) for o in out] == [(0.0, 2.0), (2.0, 4.0)]
    out = oracle.simulate_admission([0.0, 0.5], [frag, frag], [2.0, 2.0], "sensitivity", 1024, 1.5, 4,
                                    slowed=True, background=bg)
    assert [(o["admit"], o["end"]) for o in out] == [(0.0, 4.0), (4.0, 8.0)]
    assert out[1]["corunners"] == ()
    # occupancy: 0.25 + 0.25 + 0.5 reaches 1, so the occupancy rule serialises too
    out = oracle.simulate_admission([0.0, 0.5], [frag, frag], [2.0, 2.0], "usher", 1024, 1.5, 4,
                                    background=bg)
    assert [(o["admit"], o["end"]) for o in out] == [(0.0, 2.0), (2.0, 4.0)]

# ------------------------------------------------ discrete-event serving model
def _sim_jobs(n, rng, nbytes=1000):
    kinds = [_job([1.0 + 2.0 * rng.random(), 1.0], [rng.random(), 0.0], nbytes=nbytes, occ=0.4)
             for _ in range(3)]
    return [kinds[int(rng.integers(0, 3))] for _ in range(n)]


def test_simulator_single_slot_is_the_fifo_queue_recursion():
    """One slot, naive admission: the textbook single-server FIFO recursion
    end_i = max(arrival_i, end_{i-1}) + service_i (Lindley)."""
    rng = np.random.default_rng(3)
    n = 400
    arr = np.cumsum(rng.exponential(1.0, n))
    svc = rng.exponential(0.9, n)
    out = oracle.simulate_admission(list(arr), _sim_jobs(n, rng), list(svc), "naive", 1 << 30, 1.5, 1)
    end = 0.0
    for i in range(n):
        start = max(arr[i], end)
        end = start + svc[i]
        assert out[i]["admit"] == pytest.approx(start) and out[i]["end"] == pytest.approx(end)
        assert out[i]["slot"] == 0


def test_simulator_invariants():
    """FIFO without bypass, slots and memory never exceeded, unbounded
    sensitivity equal to naive, and Little's law on the whole trace
    (time-average number in the system = sum of sojourn times / horizon)."""
    rng = np.random.default_rng(11)
    n = 300
    arr = list(np.cumsum(rng.exponential(0.2, n)))
    svc = list(rng.exponential(1.0, n))
    jobs = _sim_jobs(n, rng, nbytes=3000)
    budget, slots = 10000, 4
    for pol, bound in (("naive", 1.5), ("usher", 1.5), ("sensitivity", 1.6), ("sensitivity", 2.5)):
        out = oracle.simulate_admission(arr, jobs, svc, pol, budget, bound, slots)
        adm = [o["admit"] for o in out]
        assert all(a2 >= a1 for a1, a2 in zip(adm, adm[1:]))            # FIFO, no bypass
        assert all(o["admit"] >= t for o, t in zip(out, arr))
        for i, o in enumerate(out):                                      # state at each admission
            live = [j for j in range(n) if out[j]["admit"] <= o["admit"] < out[j]["end"]]
            assert len(live) <= slots
            assert sum(jobs[j]["bytes"] for j in live) <= budget
            if pol == "sensitivity" and o["corunners"]:
                group = [jobs[j] for j in o["corunners"]] + [jobs[i]]
                assert all(oracle.predicted_slowdown_rw(group[g], group[:g] + group[g + 1:]) <= bound
                           for g in range(len(group)))
        horizon = max(o["end"] for o in out)
        events = sorted([(t, 1) for t in arr] + [(o["end"], -1) for o in out])
        area, level, last = 0.0, 0, 0.0
        for t, d in events:
            area += level * (t - last)
            level, last = level + d, t
        assert area / horizon == pytest.approx(sum(o["end"] - t for o, t in zip(out, arr)) / horizon)
    big = 1 << 40
    a = oracle.simulate_admission(arr, jobs, svc, "naive", big, 1.5, 8)
    b = oracle.simulate_admission(arr, jobs, svc, "sensitivity", big, math.inf, 8)
    assert a == b


def test_simulator_hand_case_and_slowed_service():
    """Two requests that predict 3x beside each other: sensitivity admission
    with bound 1.5 runs them one after the other, naive runs them together
    (and, with slowed service, the second takes 3x its time)."""
    frag = _job([3.0, 1.0], [1.0, 0.0], nbytes=1, occ=0.4)
    out = oracle.simulate_admission([0.0, 0.5], [frag, frag], [2.0, 2.0], "sensitivity", 1024, 1.5, 4)
    assert [(o["admit"], o["end"]) for o in out] == [(0.0, 2.0), (2.0, 4.0)]
    out = oracle.simulate_admission([0.0, 0.5], [frag, frag], [2.0, 2.0], "naive", 1024, 1.5, 4, slowed=True)
    assert [(o["admit"], o["end"]) for o in out] == [(0.0, 2.0), (0.5, 6.5)]
    assert out[1]["corunners"] == (0,)
    with pytest.raises(ValueError):
        oracle.simulate_admission([0.0], [_job([1, 1], [0, 0], nbytes=2000)], [1.0], "naive", 1024, 1.5, 4)


def test_first_fit_arena():
    ar = oracle.FirstFitArena(4096)
    a = ar.alloc(100)
    b = ar.alloc(1000)
    c = ar.alloc(256)
    assert (a, b, c) == (0, 256, 1280)                  # 256-byte granules, lowest fit
    ar.release(b, 1000)
    assert ar.largest_free() == 4096 - 1536
    assert ar.alloc(512) == 256                           # reuses the hole first
    ar.release(a, 100)
    ar.release(c, 256)
    ar.release(256, 512)
    assert ar.free == [(0, 4096)] and ar.alloc(5000) is None
