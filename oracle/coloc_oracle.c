/*
 * CPU oracle for the stressor / victim kernels.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * statement of what every kernel of the colocation suite must produce.  It
 * shares no code, header, table or constant generator with the device library
 * and must never be linked into it; only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load it.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC (the
 * contraction switch matters: the triad is defined with two roundings).
 *
 * The paper (Elvinger et al., "Understanding GPU Resource Interference One
 * Level Deeper", SoCC'25) describes its microbenchmarks only in prose:
 *   - copy kernel: repeatedly copies an input array to an output array
 *     (Section 3, Pitfall 2; Section 4.3);
 *   - compute kernel: iterated independent element-wise FP32 (or FP64)
 *     multiplies with a knob for instruction-level parallelism (Section 3,
 *     Pitfall 1; Sections 4.4.2 and 4.4.3);
 *   - shared-memory kernel: loads and stores an array inside shared memory at
 *     a stride that sets the bank-conflict degree (Section 4.4.1).
 * The exact arithmetic below (triad formula, FMA chains, checksums, pointer
 * chase, quantizers) follows the workload definitions the suite is built to;
 * every reading of a point the paper leaves open is listed in the design
 * notes and repeated next to the function that takes it.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Triad (memory-bandwidth stressor and victim).
 * a[i] = b[i] + 3.0f * c[i] in FP32 with two roundings: the product is
 * rounded to FP32, then the sum is.  No fused multiply-add. */
void or_triad_f32(const float* b, const float* c, float* a, uint64_t n) {
  for (uint64_t i = 0; i < n; ++i) {
    float t = 3.0f * c[i];
    a[i] = b[i] + t;
  }
}

/* The same triad split over `threads` host threads, each taking one
 * contiguous share of the elements (the CPU baseline runs the oracle on
 * every core of the host).  Element-wise, so the result does not depend on
 * the thread count. */
struct triad_share {
  const float* b;
  const float* c;
  float* a;
  uint64_t lo, hi;
};

static void* triad_worker(void* arg) {
  const struct triad_share* s = (const struct triad_share*)arg;
  or_triad_f32(s->b + s->lo, s->c + s->lo, s->a + s->lo, s->hi - s->lo);
  return NULL;
}

int or_triad_f32_mt(const float* b, const float* c, float* a, uint64_t n, int threads) {
  if (threads < 1) threads = 1;
  if (threads > 1024) threads = 1024;
  pthread_t tid[1024];
  struct triad_share sh[1024];
  int started = 0;
  for (int t = 0; t < threads; ++t) {
    sh[t].b = b;
    sh[t].c = c;
    sh[t].a = a;
    sh[t].lo = n * (uint64_t)t / (uint64_t)threads;
    sh[t].hi = n * (uint64_t)(t + 1) / (uint64_t)threads;
    if (t == 0) continue;  /* the calling thread takes share 0 */
    if (pthread_create(&tid[t], NULL, triad_worker, &sh[t]) != 0) break;
    started = t;
  }
  triad_worker(&sh[0]);
  for (int t = 1; t <= started; ++t) pthread_join(tid[t], NULL);
  /* shares whose thread could not start run here */
  for (int t = started + 1; t < threads; ++t) triad_worker(&sh[t]);
  return started + 1;
}

/* Sum of the raw 32-bit patterns, modulo 2**64: an order-independent
 * checksum, so any summation order on the device must match it exactly. */
uint64_t or_bitsum_u32(const uint32_t* w, uint64_t n) {
  uint64_t s = 0;
  for (uint64_t i = 0; i < n; ++i) s += (uint64_t)w[i];
  return s;
}

/* Sum of 32-bit words modulo 2**32 over w[lo:hi]. */
uint32_t or_sum_u32_mod32(const uint32_t* w, uint64_t lo, uint64_t hi) {
  uint32_t s = 0;
  for (uint64_t i = lo; i < hi; ++i) s += w[i];
  return s;
}

/* Exact sum of FP32 values, returned rounded to FP64.
 * Every finite FP32 value is an integer multiple of 2**-149 with magnitude
 * below 2**128, so x * 2**149 is an integer below 2**277.  The sum is kept as
 * a 384-bit two's-complement integer (six 64-bit limbs), which cannot
 * overflow for n < 2**100 terms.  Non-finite inputs return NaN. */
#define OR_LIMBS 6
static void limbs_add_shifted(uint64_t* acc, uint64_t m, int shift, int neg) {
  /* add (or subtract) m << shift */
  uint64_t add[OR_LIMBS];
  memset(add, 0, sizeof(add));
  int word = shift / 64, bit = shift % 64;
  add[word] = m << bit;
  if (bit && word + 1 < OR_LIMBS) add[word + 1] = m >> (64 - bit);
  if (neg) { /* two's complement negate */
    uint64_t carry = 1;
    for (int k = 0; k < OR_LIMBS; ++k) {
      uint64_t v = ~add[k];
      add[k] = v + carry;
      carry = (carry && add[k] == 0) ? 1 : 0;
    }
  }
  uint64_t carry = 0;
  for (int k = 0; k < OR_LIMBS; ++k) {
    uint64_t s = acc[k] + add[k];
    uint64_t c1 = s < acc[k];
    uint64_t s2 = s + carry;
    uint64_t c2 = s2 < s;
    acc[k] = s2;
    carry = c1 | c2;
  }
}

double or_sum_f32_exact(const float* a, uint64_t n) {
  uint64_t acc[OR_LIMBS];
  memset(acc, 0, sizeof(acc));
  for (uint64_t i = 0; i < n; ++i) {
    float x = a[i];
    if (!isfinite(x)) return NAN;
    if (x == 0.0f) continue;
    uint32_t bits;
    memcpy(&bits, &x, 4);
    int neg = bits >> 31;
    int e = (bits >> 23) & 0xFF;
    uint64_t m = bits & 0x7FFFFF;
    int shift; /* x = m * 2**(shift - 149) */
    if (e == 0) shift = 0;
    else { m |= 0x800000; shift = e - 1; }
    limbs_add_shifted(acc, m, shift, neg);
  }
  /* convert: value = signed(acc) * 2**-149 */
  int neg = (acc[OR_LIMBS - 1] >> 63) & 1;
  if (neg) {
    uint64_t carry = 1;
    for (int k = 0; k < OR_LIMBS; ++k) {
      uint64_t v = ~acc[k];
      acc[k] = v + carry;
      carry = (carry && acc[k] == 0) ? 1 : 0;
    }
  }
  long double s = 0.0L;
  for (int k = OR_LIMBS - 1; k >= 0; --k) s = s * 18446744073709551616.0L + (long double)acc[k];
  double r = (double)ldexpl(s, -149);
  return neg ? -r : r;
}

/* ------------------------------------------------------------------------ */
/* VALU chain: x <- fma(x, a, b) repeated `steps` times for each start value.
 * fmaf is the correctly rounded fused multiply-add of C99, the same
 * single-rounding operation as the device's FP32 FMA. */
void or_fma_chain_f32(const float* x0, uint64_t n, float a, float b, uint64_t steps,
                      float* out) {
  for (uint64_t i = 0; i < n; ++i) {
    float x = x0[i];
    for (uint64_t k = 0; k < steps; ++k) x = fmaf(x, a, b);
    out[i] = x;
  }
}

/* FP64 pipeline chain (the paper's FP64 compute kernel, Section 4.4.3):
 * x <- x * a, rounded to binary64 each step (one IEEE multiply). */
void or_dmul_chain(const double* x0, uint64_t n, double a, uint64_t steps, double* out) {
  for (uint64_t i = 0; i < n; ++i) {
    double x = x0[i];
    for (uint64_t k = 0; k < steps; ++k) x = x * a;
    out[i] = x;
  }
}

/* ------------------------------------------------------------------------ */
/* Pointer chase: follow next[] `hops` times from each start index. */
void or_chase_u32(const uint32_t* next, uint64_t n, const uint64_t* starts, uint64_t nchains,
                  uint64_t hops, uint32_t* end) {
  (void)n;
  for (uint64_t c = 0; c < nchains; ++c) {
    uint32_t i = (uint32_t)starts[c];
    for (uint64_t h = 0; h < hops; ++h) i = next[i];
    end[c] = i;
  }
}

/* 1 if next[] is a permutation of 0..n-1 made of exactly one cycle, else 0. */
int or_is_single_cycle(const uint32_t* next, uint64_t n) {
  if (n == 0) return 0;
  uint8_t* seen = (uint8_t*)calloc(n, 1);
  if (!seen) return -1;
  uint64_t i = 0, steps = 0;
  int ok = 1;
  do {
    if (next[i] >= n || seen[i]) { ok = 0; break; }
    seen[i] = 1;
    i = next[i];
    ++steps;
  } while (i != 0 && steps <= n);
  if (ok && steps != n) ok = 0;
  free(seen);
  return ok;
}

/* ------------------------------------------------------------------------ */
/* LDS loop checksum of one wave for one pass.
 * Window: `nvec` vectors of `vw` 32-bit words (vw in {1, 2, 4}).  At step k
 * (0 <= k < nvec) lane l touches vector (l * stride + k) mod nvec, so over a
 * pass each lane visits every vector once.  Returns the sum, mod 2**32, of
 * every word read by the 64 lanes. */
uint32_t or_lds_wave_pass_sum(const uint32_t* window, uint32_t nvec, uint32_t vw,
                              uint32_t stride) {
  uint32_t s = 0;
  for (uint32_t lane = 0; lane < 64; ++lane)
    for (uint32_t k = 0; k < nvec; ++k) {
      uint32_t v = (uint32_t)(((uint64_t)lane * stride + k) % nvec);
      for (uint32_t j = 0; j < vw; ++j) s += window[(uint64_t)v * vw + j];
    }
  return s;
}

/* ------------------------------------------------------------------------ */
/* BF16: the FP32 value nearest to x whose low 16 bits are zero, ties to the
 * candidate with an even 16-bit code (IEEE round-to-nearest-even).  NaN maps
 * to the quiet NaN 0x7FC0 with x's sign; infinities are kept; values whose
 * nearest candidate overflows round to infinity as IEEE prescribes. */
static double bf16_value(uint16_t h) {
  uint32_t bits = (uint32_t)h << 16;
  float f;
  memcpy(&f, &bits, 4);
  return (double)f;
}

void or_f32_to_bf16(const float* x, uint64_t n, uint16_t* out) {
  for (uint64_t i = 0; i < n; ++i) {
    float v = x[i];
    uint32_t bits;
    memcpy(&bits, &v, 4);
    if (isnan(v)) { out[i] = (uint16_t)(((bits >> 16) & 0x8000) | 0x7FC0); continue; }
    uint16_t lo = (uint16_t)(bits >> 16);         /* truncation toward zero */
    if ((bits & 0xFFFF) == 0) { out[i] = lo; continue; }
    uint16_t hi = (uint16_t)(lo + 1);              /* next code away from zero */
    double dv = (double)v, dlo = bf16_value(lo);
    double dhi = ((hi & 0x7FFF) == 0x7F80) ? (dv > 0 ? 1.0 : -1.0) * ldexp(1.0, 128)
                                           : bf16_value(hi);
    double elo = fabs(dv - dlo), ehi = fabs(dhi - dv);
    uint16_t pick;
    if (elo < ehi) pick = lo;
    else if (ehi < elo) pick = hi;
    else pick = (lo & 1) ? hi : lo;
    out[i] = pick;
  }
}

/* ------------------------------------------------------------------------ */
/* FP8 E4M3 (OCP 8-bit floating point specification, "E4M3FN"): 1 sign bit,
 * 4 exponent bits with bias 7, 3 mantissa bits, no infinities, the single
 * NaN pattern S.1111.111, largest finite magnitude 448 (S.1111.110),
 * subnormals m * 2**-9. */
double or_e4m3_decode(uint8_t code) {
  int s = code >> 7, e = (code >> 3) & 0xF, m = code & 7;
  if (e == 0xF && m == 7) return NAN;
  double mag = (e == 0) ? ldexp((double)m, -9) : ldexp(1.0 + m / 8.0, e - 7);
  return s ? -mag : mag;
}

/* Encode with round-to-nearest-even and saturation to +-448 (values beyond
 * the largest finite magnitude, including infinities, become +-448).
 * Plain search: the nearest of the 127 non-negative finite magnitudes, ties
 * to the even code.  NaN becomes 0x7F with x's sign. */
void or_f32_to_e4m3(const float* x, uint64_t n, uint8_t* out) {
  double mags[127];
  for (int c = 0; c < 127; ++c) mags[c] = or_e4m3_decode((uint8_t)c);
  for (uint64_t i = 0; i < n; ++i) {
    float v = x[i];
    uint8_t sign = signbit(v) ? 0x80 : 0;
    if (isnan(v)) { out[i] = sign | 0x7F; continue; }
    double a = fabs((double)v);
    if (a >= 448.0) { out[i] = sign | 0x7E; continue; }
    /* binary search for the largest code with mags[c] <= a */
    int lo = 0, hi = 126;
    while (lo < hi) {
      int mid = (lo + hi + 1) / 2;
      if (mags[mid] <= a) lo = mid; else hi = mid - 1;
    }
    int c = lo;
    if (mags[c] != a && c < 126) {
      double dlo = a - mags[c], dhi = mags[c + 1] - a;
      if (dhi < dlo || (dhi == dlo && (c & 1))) c = c + 1;
    }
    out[i] = sign | (uint8_t)c;
  }
}
