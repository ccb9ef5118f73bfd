/*
 * coloc.h -- C ABI of libcoloc.so, the MI355X (gfx950) resource-stressor
 * suite and victim-colocation harness.
 *
 * What it measures follows Elvinger et al., "Understanding GPU Resource
 * Interference One Level Deeper" (SoCC'25):
 *   - one microbenchmark per shared GPU resource, each holding a constant
 *     level of interference for the whole life of the colocated workload
 *     (Section 4.1);
 *   - the workload's slowdown colocated versus in isolation (Section 4.3,
 *     cache-pollution experiment), per resource and per intensity, as the
 *     sensitivity profile a kernel-level interference estimator consumes
 *     (Section 5.1);
 *   - the stressor's own utilisation as a fraction of the resource's peak
 *     (Section 2.2 metrics; Tables 1-3).
 * Intra-CU colocation is two HIP streams; the CU-partitioned (inter-CU)
 * mode, the paper's green-context setting (Section 4.1), uses CU-masked
 * streams.
 *
 * Conventions for every call:
 *   - Returns ci_status_t; never throws, never exits.  On error,
 *     ci_last_error() returns a thread-local message (valid until the next
 *     call on the same thread).
 *   - "device pointer" = memory of the context's GPU, allocated by the caller
 *     (e.g. torch) unless stated; the library never frees it.
 *   - `stream` arguments are hipStream_t values passed as void*.  The call's
 *     work is ordered after work already queued on `stream`, and `stream`
 *     waits for the call's results.  NULL means "no ordering": the caller
 *     must have finished its own prior work (the legacy null stream is never
 *     used, because it would serialise against the CU-masked streams).
 *   - Device timestamps are the GPU's constant-rate wall clock
 *     (ci_device_info_t.wall_clock_khz ticks per millisecond).
 *   - A context is used by one host thread at a time.
 */
#ifndef COLOC_H
#define COLOC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ci_status {
  CI_OK = 0,
  CI_ERR_INVALID_ARG = 1,  /* bad pointer, size, enum, intensity or option */
  CI_ERR_HIP = 2,          /* a HIP runtime call failed (message names it)  */
  CI_ERR_OOM = 3,          /* device or host allocation failed / budget    */
  CI_ERR_TIMEOUT = 4,      /* a stressor hit its in-kernel deadline, or did
                              not start within the start timeout           */
  CI_ERR_UNSUPPORTED = 5,  /* combination not implemented on this device   */
  CI_ERR_BUSY = 6,         /* context already has a stressor on that slot  */
  CI_ERR_DRAIN = 7         /* a stressor kernel did not exit within its
                              deadline + 5 s after the stop request; the
                              context launches no further stressors        */
} ci_status_t;

/* Shared resources with one stressor each (paper Section 4: block scheduler
 * 4.2; L2 capacity and memory bandwidth 4.3; shared memory 4.4.1; issue
 * (IPC) 4.4.2; compute pipelines 4.4.3), mapped to CDNA4 units. */
typedef enum ci_resource {
  CI_RES_HBM = 0,        /* array streaming: triad a = b + 3c, or a CI_HBM_* mix */
  CI_RES_L2 = 1,         /* every WG re-reads one region sized for each XCD's L2 */
  CI_RES_MALL = 2,       /* array streaming over a footprint that misses L2 and
                            fits the Infinity Cache                            */
  CI_RES_VL1D = 3,       /* ... a region that fits the per-CU vector L1        */
  CI_RES_LDS = 4,        /* LDS copy loop with a stride (bank-conflict) knob   */
  CI_RES_VALU_F32 = 5,   /* FP32 FMA chains with an ILP knob                   */
  CI_RES_MFMA_F32 = 6,   /* matrix-core loops, FP32 inputs                     */
  CI_RES_MFMA_BF16 = 7,  /* ... BF16 inputs                                    */
  CI_RES_MFMA_FP8 = 8,   /* ... FP8 E4M3 inputs                                */
  CI_RES_PTRCHASE = 9,   /* dependent loads through a random cycle             */
  CI_RES_DISPATCH = 10,  /* stream of empty 64-thread work-groups              */
  CI_RES_OCCUPANCY = 11, /* sleeping WGs that hold LDS / wave slots (Sec. 4.2)  */
  CI_RES_VALU_F64 = 12,  /* FP64 multiply chains with an ILP knob (Sec. 4.4.3) */
  CI_RES_COUNT = 13
} ci_resource_t;

typedef enum ci_dtype { CI_DT_F32 = 0, CI_DT_BF16 = 1, CI_DT_FP8E4M3 = 2 } ci_dtype_t;

typedef enum ci_victim_kind {
  CI_VICTIM_TRIAD_F32 = 0, /* a = b + 3c (FP32), `passes` sweeps per launch    */
  CI_VICTIM_GEMM = 1,      /* C = s_a s_b A B^T, FP32 accumulate and output    */
  CI_VICTIM_GEMV = 2       /* y = W x, BF16 in, FP32 accumulate and output     */
} ci_victim_kind_t;

typedef enum ci_placement {
  CI_PLACE_SHARED = 0,     /* victim may use every CU (intra-CU colocation)    */
  CI_PLACE_DISJOINT = 1    /* victim confined to the CUs the stressor lacks    */
} ci_placement_t;

typedef struct ci_ctx ci_ctx_t;
typedef struct ci_stressor ci_stressor_t;

/* ---------------------------------------------------------------- device */
typedef struct ci_device_info {
  int device;
  int num_cus;              /* compute units visible (256 on MI355X)        */
  int num_xcds;             /* accelerator complex dies (8)                  */
  int wave_size;            /* 64                                            */
  int clock_khz;            /* peak engine clock reported by the runtime     */
  int wall_clock_khz;       /* device timestamp rate                          */
  uint64_t lds_bytes_per_cu;
  uint64_t l2_bytes_per_xcd;
  uint64_t hbm_bytes;
  char arch[64];            /* gcnArchName, e.g. "gfx950:sramecc+:xnack-"    */
  /* peak denominators used for %-of-peak (published figures for MI355X,
   * or, where none is published, per-clock derivations: see
   * ci_peak_for()).                                                          */
  double peak[CI_RES_COUNT];
} ci_device_info_t;

/* Create a context on HIP device `device`: reads device properties, builds
 * the CU-mask layout and allocates the small internal scratch (checksum
 * partials, pinned control block).  *out owned by the library. */
ci_status_t ci_init(int device, ci_ctx_t** out);
/* Destroy a context; stops nothing: every stressor must be stopped first
 * (CI_ERR_BUSY otherwise).  NULL is a no-op. */
ci_status_t ci_shutdown(ci_ctx_t* ctx);
const char* ci_last_error(void);
ci_status_t ci_device_info(ci_ctx_t* ctx, ci_device_info_t* out);

/* Peak of resource r in its own unit: bytes/s for HBM, L2, MALL, VL1D and
 * LDS; flop/s for VALU and MFMA (for VALU_F64 one multiply = one flop, so its
 * peak is half the FP64 FMA rate); work-groups/s for DISPATCH; hops/s for the
 * chase (no peak: 0); OCCUPANCY has no rate (0).  HBM and the matrix cores
 * take MI355X's published figures; L2, vL1D and the vector ALUs bytes or
 * flops per clock times units times the 2.4 GHz engine clock; the Infinity
 * Cache and the LDS, for which no figure describes CDNA4, a ceiling measured
 * on MI355X (Infinity Cache 7.65 TB/s, the best streaming rate any launch
 * shape reached; LDS 117 B/clk per CU, a conflict-free 16-byte copy). */
ci_status_t ci_peak_for(ci_ctx_t* ctx, ci_resource_t r, double* peak);

/* ------------------------------------------------------------ CU masks */
/* Intensity x in [0, 1] -> k = 8 * round(32 * x) CUs (num_xcds *
 * round(num_cus / num_xcds * x) in general): whole steps of one CU on every
 * XCD, since work-groups are dealt to the XCDs round-robin and a queue whose
 * mask leaves an XCD empty cannot be created.  CU-mask bit b selects CU b/8
 * of XCD b mod 8, so the mask is bits 0..k-1.  mask: 8 uint32 words as
 * hipExtStreamCreateWithCUMask reads them.  complement != 0 returns the other
 * num_cus - k CUs (the disjoint-placement victim mask).  *ncu receives the
 * number of CUs in the returned mask. */
ci_status_t ci_cu_mask(ci_ctx_t* ctx, float intensity, int complement, uint32_t mask[8],
                       int* ncu);

/* Placement probe (the AMD analog of the paper's per-block SM-ID print,
 * Section 4.2 footnote): launches `nwg` 64-thread work-groups on a stream
 * restricted to `mask` (NULL = all CUs; CI_ERR_INVALID_ARG if the mask
 * leaves an XCD without CUs); work-group i writes its hardware
 * location to out_loc[i] (device pointer, nwg uint32):
 *   bits 0-3 CU id, bit 4 shader array, bits 5-6 shader engine, bits 8-11 XCD.
 * Synchronous. */
ci_status_t ci_probe_placement(ci_ctx_t* ctx, const uint32_t* mask, uint32_t nwg,
                               uint32_t* out_loc);

/* Queue-pair check counters.  Two hardware queues can slow each other's
 * kernels although the kernels share no CU (the command-processor side of
 * the paper's block-scheduler interference, Section 4.2), and on MI355X
 * whether two queues do so depends on where the driver placed them.  Before
 * the first colocated measurement of a (victim queue, stressor queue) pair in
 * each call, measure_sensitivity and measure_decode run the victim alone and beside an
 * idle kernel on the stressor's queue (sleeping work-groups on the
 * stressor's CUs: one of 256 threads per CU on shared CUs, the stressor's own
 * launch shape on disjoint CUs); if the idle kernel slows the victim by more
 * than 5 %, a queue is replaced (the stressor's and the victim's in turn, at
 * most 7 times).  A victim queue is first qualified: measured alone against
 * two fresh queues with the same mask, the fastest kept (a queue can also be
 * slow on its own).  serve_run_background checks each slot stream against
 * its stressor's queue the same way (with a probe triad as the victim).
 *   *checks: pairs checked; *replaced: queues replaced (by either step);
 *   *unresolved: pairs
 *   still above 5 % after the last replacement (measured as placed). */
ci_status_t ci_queue_stats(ci_ctx_t* ctx, uint32_t* checks, uint32_t* replaced,
                           uint32_t* unresolved);

/* ----------------------------------------------------------- stressors */
/* Per-work-group record written by every stressor work-group at exit
 * (device memory inside the caller's workspace, after the 2304 bytes of
 * control words). */
typedef struct ci_wg_record {
  uint64_t t_start;  /* device wall clock at WG start                      */
  uint64_t t_end;    /* device wall clock at WG exit                       */
  uint64_t work;     /* passes completed (per resource unit, see below)    */
  uint64_t check;    /* checksum accumulated by the WG (resource specific) */
  uint32_t loc;      /* hardware location, encoded as in ci_probe_placement */
  uint32_t flags;    /* bit 0: exited on its deadline; bit 1: saw stop     */
  uint64_t pad;
} ci_wg_record_t;    /* 48 bytes */

/* Traffic mixes of the streaming stressors (the knob of HBM and MALL).  The
 * paper's bandwidth stressor streams large arrays through memory (Section
 * 3, Pitfall 2; Section 4.3, Table 1); the mix sets the read/write
 * proportion of that stream, since bandwidth and a co-runner's slowdown both
 * depend on it.  Per element i < n (4-byte words, every element once per
 * pass):
 *   CI_HBM_TRIAD  a[i] = b[i] + 3 c[i] in FP32, rounded after the product
 *                 and after the sum; 2 reads : 1 write, 12 B (default)
 *   CI_HBM_READ   reads b[i] and c[i]; nothing is stored; each work-group's
 *                 record.check is the sum of the words it read mod 2^32, so
 *                 the checksum over all records, mod 2^32, is passes x
 *                 sum_i (b[i] + c[i]) as uint32 words; 8 B
 *   CI_HBM_COPY   a[i] = b[i] (bit copy); 1 : 1, 8 B
 *   CI_HBM_WRITE  a[i] = the bits of lo32(i) * 0x9E3779B1 mod 2^32; 4 B    */
#define CI_HBM_TRIAD 1u
#define CI_HBM_READ 2u
#define CI_HBM_COPY 3u
#define CI_HBM_WRITE 4u

typedef struct ci_stressor_opts {
  /* Resource-specific operands (device pointers, caller-owned):
   *   HBM, MALL:  src0 = b, src1 = c, dst = a   (FP32, n elements; only the
   *               arrays the traffic mix touches are required; n <= 2^32 for
   *               the write-only mix).  HBM: arrays far larger than the
   *               256 MB Infinity Cache; MALL: a footprint larger than the
   *               L2s (4 MB per XCD) that fits the Infinity Cache.  Each XCD
   *               slot streams its own eighth of the arrays.
   *   L2/VL1D:    src0 = region (uint32, n words)
   *   LDS:        src0 = window words (uint32, 8192 = 32 KiB)
   *   VALU_F32:   dst  = final chain values (FP32, grid*threads*knob)
   *   VALU_F64:   dst  = final chain values (FP64, grid*threads*knob); the
   *               multiplier is (double)fa
   *   MFMA_*:     src0 = A tile (32 x K), src1 = B tile (K x 32), row-major,
   *               element type F32 / BF16 / E4M3 with K = 2 / 16 / 64;
   *               dst = per-wave accumulator tiles (FP32, waves*knob*32*32)
   *   PTRCHASE:   src0 = next[] (uint32, n entries, one cycle),
   *               dst = end index per chain (uint32, grid*threads*knob)
   *   DISPATCH:   dst = uint64 counter of work-groups executed (may be NULL
   *               for the empty-kernel timing form)
   *   OCCUPANCY:  none                                                       */
  const void* src0;
  const void* src1;
  void* dst;
  uint64_t n;
  uint32_t wg_per_cu;    /* work-groups per masked CU; 0 = resource default  */
  uint32_t threads;      /* threads per work-group; 0 = resource default     */
  uint32_t knob;         /* VALU_F32/F64: ILP chains per lane (1,2,4,8); LDS: stride
                            in vectors; MFMA: independent accumulators (1-4);
                            HBM, MALL: traffic mix CI_HBM_* (0 = triad for
                            HBM, read-only for MALL);
                            PTRCHASE: chains per lane (1-8); OCCUPANCY: LDS
                            KiB held per WG; 0 = default                     */
  uint32_t vec;          /* LDS: vector width in 32-bit words (1, 2, 4);
                            HBM: 0 = streaming (non-temporal) accesses,
                            1 = ordinary cached accesses; MALL: always
                            cached                                          */
  uint64_t passes;       /* 0 = run until stressor_stop; > 0 = exactly this
                            many passes per work-group, then exit            */
  uint64_t iters;        /* VALU: FMA steps per pass (default 4096); MFMA:
                            MFMAs per accumulator per pass (default 1024);
                            PTRCHASE: hops per pass (default 65536);
                            DISPATCH: work-groups per launch (default 1e6)   */
  float fa, fb;          /* VALU chain x <- fma(x, fa, fb)                   */
  uint32_t deadline_ms;  /* in-kernel safety deadline, 0 = 2000 ms           */
  uint32_t duty;         /* percent of time the stressor is active (1..100;
                            0 = 100): after each pass (HBM, MALL: each round
                            of chunks) a wave idles for (100/duty - 1) times
                            the time the pass took, so the unit sees duty% of
                            the load on every masked CU.  Ignored by DISPATCH /
                            OCCUPANCY */
  uint32_t chunk;        /* HBM, MALL: 16-byte accesses per lane and stream in
                            one wave-chunk (1, 2 or 4; 0 = 4): a wave-chunk is
                            256 * chunk elements                            */
  uint32_t access;       /* LDS: CI_LDS_COPY (0; each vector is loaded from one
                            window and stored to the other, the paper's strided
                            copy, Section 4.4.1) or CI_LDS_LOAD (loads only:
                            the read path at full rate).  Must be 0 for every
                            other resource                                  */
} ci_stressor_opts_t;

#define CI_LDS_COPY 0u
#define CI_LDS_LOAD 1u

typedef struct ci_stressor_report {
  int resource;
  int ncu;                  /* CUs in the stressor's mask                    */
  uint32_t grid;            /* work-groups launched                          */
  uint32_t wg_reported;     /* records with t_end != 0                       */
  uint64_t t_first_start;   /* min record t_start                            */
  uint64_t t_last_start;    /* max record t_start                            */
  uint64_t t_first_end;     /* min record t_end                              */
  uint64_t t_last_end;      /* max record t_end                              */
  double window_ns;         /* t_last_end - t_first_start in ns              */
  double kernel_ns;         /* event time of the launch(es)                  */
  uint64_t work;            /* sum of record work                            */
  double units;             /* algorithmic bytes / flops / WGs / hops        */
  double achieved;          /* units / window seconds                        */
  double pct_of_peak;       /* 100 * achieved / peak (0 if no peak)          */
  uint64_t checksum;        /* sum of record checks mod 2^64                 */
  int timed_out;            /* some WG exited on its deadline                */
  int distinct_cus;         /* distinct hardware CUs seen in the records     */
} ci_stressor_report_t;

/* Device bytes of workspace stressor r needs at CU fraction `intensity`
 * with options opts (NULL = defaults): 2304 bytes of control words (stop and
 * start words, the dispatch counter, one ticket line per XCD slot for the
 * streaming stressors) and one 48-byte record per work-group, the grid
 * being (work-groups per CU) x
 * (CUs at that intensity).  The count uses the 256-CU layout (exact on
 * MI355X, an upper bound on parts with fewer CUs); intensity 1 bounds every
 * intensity.  The options stay an argument because the work-groups per CU
 * (opts->wg_per_cu) set the record count.  Pure host computation.
 * CI_ERR_INVALID_ARG on a bad resource, NaN or out-of-range intensity, or
 * NULL bytes. */
ci_status_t ci_workspace_size(ci_resource_t r, float intensity, const ci_stressor_opts_t* opts,
                              size_t* bytes);

/* Start stressor r at CU fraction `intensity` (0..1, rounded as in
 * ci_cu_mask): one microbenchmark per shared resource holding a constant
 * level of interference for as long as the colocated workload runs
 * (Section 4.1); the intensity is the fraction of compute units it may use,
 * as the paper sizes its stressors by the SMs they get (Section 4.1, green
 * contexts; Section 4.3, Table 1).  The kernel runs on a
 * library-owned CU-masked stream that first waits for work already queued on
 * `stream` (which is not blocked).  With opts->passes == 0 the call returns
 * once the stressor is observed running on the device (all its work-groups
 * resident, or 50 ms elapsed), and it keeps running until stressor_stop or
 * its deadline.  With passes > 0 it returns right after the launch.
 * intensity == 0 returns a valid handle that launches nothing.  ws: device
 * workspace of ws_bytes >= ci_workspace_size(); must stay allocated until
 * stressor_stop returns.  One running stressor per context at a time:
 * CI_ERR_BUSY otherwise. */
ci_status_t stressor_launch(ci_ctx_t* ctx, ci_resource_t r, float intensity, void* stream,
                            const ci_stressor_opts_t* opts, void* ws, size_t ws_bytes,
                            ci_stressor_t** h);

/* End the constant interference started by stressor_launch (Section 4.1):
 * signal stop, wait for the kernel(s) to drain (bounded by the deadline),
 * make `stream` of the launch wait for completion, read the records and fill
 * *rep (may be NULL) with the stressor's own utilisation as a fraction of
 * the resource's peak (the paper's utilisation metrics, Section 2.2, and the
 * stressor rows of Tables 1-3).  Frees h.  Returns CI_ERR_TIMEOUT (after
 * filling rep) if a work-group hit its deadline, CI_ERR_DRAIN if the kernel
 * did not exit within the deadline + 5 s. */
ci_status_t stressor_stop(ci_stressor_t* h, ci_stressor_report_t* rep);

/* Copy the stressor's records (grid entries) to host memory; valid only
 * between the end of stressor_stop's drain and the next launch: call with
 * the same ws after stressor_stop. */
ci_status_t ci_read_records(ci_ctx_t* ctx, const void* ws, uint32_t grid, ci_wg_record_t* out);

/* -------------------------------------------------------------- victims */
typedef struct ci_victim_desc {
  int kind;              /* ci_victim_kind_t                                  */
  int dtype;             /* GEMM: F32 / BF16 / FP8E4M3; GEMV: BF16; TRIAD: F32 */
  uint64_t m, n, k;      /* TRIAD: n elements; GEMM: M, N, K; GEMV: n rows, k cols */
  const void* a;         /* TRIAD: b; GEMM: A (M x K row-major); GEMV: W (copies x n x k) */
  const void* b;         /* TRIAD: c; GEMM: B (N x K row-major); GEMV: x (k)  */
  void* out;             /* TRIAD: a (n FP32); GEMM: C (M x N FP32); GEMV: y (n FP32) */
  float scale_a, scale_b;/* FP8 dequantisation scales (ignored otherwise)     */
  uint32_t passes;       /* TRIAD sweeps per run (>= 1)                        */
  uint32_t copies;       /* GEMV weight copies rotated over runs (>= 1)        */
  uint32_t flags;        /* TRIAD: CI_VICTIM_TRIAD_IN_KERNEL or 0; 0 otherwise */
  uint32_t reserved;     /* must be 0                                         */
} ci_victim_desc_t;

/* TRIAD victim flag.  Without it the run is `passes` launches of one sweep
 * each, so every sweep reads the arrays from where a fresh launch finds
 * them.  With it the passes run inside one launch: every wave sweeps its
 * own chunks (w, w + W, ... for wave w of W) `passes` times, so a working
 * set that fits a cache level is re-read from that level -- the form of the
 * cache-pollution experiment (Section 4.3, Figure 3), whose instances keep
 * copying their own data.  Same output either way. */
#define CI_VICTIM_TRIAD_IN_KERNEL 1u

typedef struct ci_victim_result {
  double time_ns;          /* launch time from HIP events                      */
  uint64_t checksum_bits;  /* sum of the output's 32-bit patterns mod 2^64     */
  double sum_f64;          /* FP64 sum of the output (fixed reduction order)   */
  uint64_t t_begin;        /* device clock just before / after the victim      */
  uint64_t t_end;
} ci_victim_result_t;

/* Run the victim once on `stream` and wait for it: the workload whose
 * latency the paper compares alone and colocated (Section 4.1; its victims
 * are a GEMM for shared memory, Section 4.4.1, and LLM decode, dominated by
 * matrix-vector products, Sections 4.2-4.3).  One kernel launch (a triad of
 * `passes` sweeps: `passes` launches) timed with HIP events, bracketed by
 * device timestamps, followed by the output checksum.  Victim constraints: TRIAD n >= 0; GEMM K a multiple of 16 / 8 /
 * 4 elements for FP8 / BF16 / F32 (any M, N); GEMV k a multiple of 8. */
ci_status_t victim_run(ci_ctx_t* ctx, const ci_victim_desc_t* d, void* stream,
                       ci_victim_result_t* out);

/* Enqueue `count` back-to-back launches of the victim's kernel on `stream`
 * (non-NULL) and return without waiting: no events, stamps or checksums.
 * Used to keep a second workload running beside a timed victim, the way the
 * paper's estimator is validated on workload pairs (Section 5.1).  The
 * caller synchronises `stream` before reusing the buffers. */
ci_status_t victim_enqueue(ci_ctx_t* ctx, const ci_victim_desc_t* d, void* stream, uint32_t count);

/* Enqueue on `stream` (non-NULL) a one-wave kernel that writes the device
 * wall clock (ticks at ci_device_info_t.wall_clock_khz, the clock of the
 * victim and stressor stamps) to *slot, a device address.  Bracketing
 * enqueued work with two stamps shows whether it covered a timed victim's
 * window [t_begin, t_end] (Section 4.1: interference constant over the
 * victim's lifetime).  Returns without waiting. */
ci_status_t ci_stamp(ci_ctx_t* ctx, uint64_t* slot, void* stream);

/* Checksums of n FP32 values at device pointer x (stream-ordered on
 * `stream`, synchronous): bit-pattern sum mod 2^64 and FP64 sum. */
ci_status_t ci_checksum_f32(ci_ctx_t* ctx, const void* x, uint64_t n, void* stream,
                            uint64_t* bits, double* sum);

/* Per-tensor quantisation on the device (precision extension):
 *   dtype BF16: dst (uint16 codes) = round-to-nearest-even of src;
 *   dtype FP8E4M3: amax = max|src|, inv = 448/amax, scale = amax/448 (FP32),
 *     dst (uint8 codes) = E4M3FN(fl32(src * inv)), nearest-even, saturating
 *     at +-448; *scale_out = scale (1 when amax == 0).
 * Synchronous on `stream`. */
ci_status_t ci_quantize(ci_ctx_t* ctx, const void* src, uint64_t n, int dtype, void* dst,
                        float* scale_out, void* stream);

/* One matrix-core instruction per tile, D = A B + C, in FP32 accumulate:
 * the building block of the GEMM victim and the matrix-core stressors
 * (Section 4.4.3 stresses the compute pipelines; the precision extension
 * asks for each dtype's error against FP64).  The instruction set leaves
 * the accumulation inside one instruction unspecified; this call lets a
 * test characterise it.  Per tile t (device pointers, tiles contiguous):
 *   dtype F32:     A 32 x 2 FP32, B 2 x 32 FP32        (v_mfma_f32_32x32x2_f32)
 *   dtype BF16:    A 32 x 16 BF16, B 16 x 32 BF16      (v_mfma_f32_32x32x16_bf16)
 *   dtype FP8E4M3: A 32 x 64 E4M3, B 64 x 32 E4M3      (v_mfma_f32_32x32x64_f8f6f4,
 *                  OCP E4M3 for both operands, no block scales)
 * all row-major; C and D 32 x 32 FP32 row-major (D may alias C).
 * Synchronous on `stream`.  CI_ERR_INVALID_ARG on NULL pointers or a bad
 * dtype. */
ci_status_t ci_mfma_probe(ci_ctx_t* ctx, int dtype, const void* a, const void* b, const float* c,
                          float* d, uint32_t ntiles, void* stream);

/* ------------------------------------------------------- sensitivity */
/* ci_measure_opts_t.flags */
#define CI_MEASURE_NO_QUEUE_CHECK 1u  /* skip the queue-pair check (raw placement) */

typedef struct ci_measure_opts {
  uint32_t reps;         /* alone/colocated pairs per cell (default 20)       */
  uint32_t warmups;      /* victim warm-up runs per cell (default 3)          */
  int placement;         /* ci_placement_t                                    */
  uint32_t deadline_ms;  /* stressor deadline per colocated run (default 2000) */
  uint32_t flags;        /* CI_MEASURE_* bits                                 */
  /* Optional caller-owned host arrays of nr * nx * reps doubles (NULL =
   * not wanted; reps after its default is applied): the victim's time in ns
   * of every alone run and every colocated run, cell c = i * nx + j, rep r
   * at index c * reps + r.  Cells that are not measured (disjoint placement
   * at intensity 1) hold NaN. */
  double* rep_alone_ns;
  double* rep_col_ns;
} ci_measure_opts_t;

typedef struct ci_cell {
  int resource;
  float intensity;
  int ncu;
  double slowdown;            /* median(T_col) / median(T_alone)             */
  double slowdown_p10, slowdown_p90;  /* of the per-rep ratios               */
  double t_alone_ns;          /* medians                                      */
  double t_col_ns;
  double stressor_achieved;   /* mean over reps, resource units / s          */
  double stressor_pct_peak;
  int window_covered;         /* every colocated run inside the stressor window */
  int output_equal;           /* every colocated output checksum == alone      */
  int timed_out;
  int reps;
  double slowdown_ci_lo;      /* percentile-bootstrap 95 % interval of the    */
  double slowdown_ci_hi;      /* slowdown (ci_bootstrap_slowdown, 1000
                                 resamples, seed 16909 + cell index)         */
  int queue_unresolved;       /* the queue-pair check could not find a pair
                                 of queues that leave each other alone: the
                                 cell was measured as placed and may carry
                                 queue interference (see ci_queue_stats)     */
} ci_cell_t;

/* Percentile-bootstrap confidence interval of the slowdown statistic
 * median(col) / median(alone) (the sensitivity measure of Section 4.3; the
 * paper reports no interval, so this is the reading used here).  Resample r
 * (0 <= r < resamples) draws na alone times and then nc colocated times with
 * replacement; draw j of resample r uses the counter-form SplitMix64 word
 *   w_k = mix(seed + (k + 1) * 0x9E3779B97F4A7C15),  k = r * (na + nc) + j,
 * (mix = the SplitMix64 output function) and picks index w_k mod na (alone,
 * j < na) or w_k mod nc (colocated, j >= na, index j - na of that draw).
 * Medians of even counts are the mean of the middle two.  *lo and *hi are
 * the 2.5 % and 97.5 % quantiles of the resampled ratios, linearly
 * interpolated between order statistics (position q * (resamples - 1)).
 * Host arrays, caller-owned; pure host computation, no device needed.
 * CI_ERR_INVALID_ARG on NULL pointers or zero counts. */
ci_status_t ci_bootstrap_slowdown(const double* alone, uint32_t na, const double* col, uint32_t nc,
                                  uint32_t resamples, uint64_t seed, double* lo, double* hi);

/* The victim's sensitivity profile: its slowdown colocated versus alone
 * (Section 4.3, the slowdown of the cache-pollution experiment; Section 4.1,
 * constant interference over the victim's lifetime) for every shared
 * resource and intensity, the per-resource profile the paper's estimator
 * consumes (Section 5.1).  For every resource rs[i] (operands in sopts[i])
 * and intensity xs[j]: warm the victim up, then `reps` times run it alone
 * and colocated with the stressor (persistent mode), checking the window and
 * output of each colocated run; cells[i * nx + j] receives the result and,
 * when o->rep_alone_ns / rep_col_ns are given, the per-rep times.  Even repetitions
 * run alone first, odd ones colocated first (counterbalanced order).  ws: workspace large
 * enough for every listed stressor at full intensity.  Synchronous. */
ci_status_t measure_sensitivity(ci_ctx_t* ctx, const ci_victim_desc_t* d,
                                const ci_resource_t* rs, const ci_stressor_opts_t* sopts, int nr,
                                const float* xs, int nx, const ci_measure_opts_t* o, void* ws,
                                size_t ws_bytes, void* stream, ci_cell_t* cells);

/* -------------------------------------------------------- decode victim */
/* One decode step of a Llama-style decoder with random weights: the
 * stand-in for the paper's LLM decode victims (Sections 4.2-4.4), whose
 * weights and serving stack are not available.  Fig. 5 breaks one decode
 * step into its kernels; the step here can be timed kernel by kernel too.
 * Per layer, as launched:
 *   QKV      RMS norm of the residual stream, QKV GEMV, rotary embedding of
 *            queries and keys, keys and values appended to the cache;
 *   ATTN     grouped-query attention over 64-position chunks of the cache;
 *   COMBINE  merge of the chunks (softmax normalisation), BF16 out;
 *   OPROJ    output GEMV + residual;
 *   GATE_UP  RMS norm, gate/up GEMV, SiLU(gate) * up, BF16 out;
 *   DOWN     down GEMV + residual;
 * after the last layer LM_HEAD: final RMS norm and the vocabulary GEMV.
 * BF16 weights, cache and GEMV inputs; FP32 accumulation, residual stream
 * and GEMV outputs. */
typedef enum ci_decode_kernel {
  CI_DK_QKV = 0, CI_DK_ATTN = 1, CI_DK_ATTN_COMBINE = 2, CI_DK_OPROJ = 3, CI_DK_GATE_UP = 4,
  CI_DK_DOWN = 5, CI_DK_LM_HEAD = 6, CI_DK_COUNT = 7
} ci_decode_kernel_t;

/* ci_decode_desc_t.flags */
#define CI_DECODE_KERNEL_TIMES 1u  /* start/stop events on every launch      */
#define CI_DECODE_GRAPH 2u         /* replay the launches as a HIP graph,
                                      captured on first use per descriptor
                                      contents and context length bucket    */

typedef struct ci_decode_config {
  uint32_t hidden;     /* model width; multiple of 8                          */
  uint32_t n_q;        /* query heads                                          */
  uint32_t n_kv;       /* key/value heads; n_q / n_kv in 1..16                 */
  uint32_t head_dim;   /* 128 or 256                                           */
  uint32_t ffn;        /* MLP width; multiple of 8                             */
  uint32_t vocab;      /* output rows; 0 = no vocabulary projection            */
  uint32_t layers;     /* >= 1                                                 */
  uint32_t batch;      /* sequences per step, 1..8                             */
  uint32_t max_ctx;    /* cache positions per sequence                         */
  float eps;           /* RMS-norm epsilon                                     */
  float rope_base;     /* rotary base (pair i turns by pos * base^(-2i/head_dim)) */
} ci_decode_config_t;

/* Element offsets (BF16 elements) into the weight arena, and sizes.  Layer
 * l's tensors sit at the layer-0 offset + l * layer_stride.  Every offset is
 * a multiple of 64 elements (128 bytes).
 *   g_attn, g_mlp, g_final: hidden gains
 *   w_qkv: (n_q + 2 n_kv) * head_dim rows x hidden (query heads, key heads,
 *          value heads; head h at rows h * head_dim ..)
 *   w_o: hidden x (n_q * head_dim)     w_gu: 2 ffn x hidden (gate, then up)
 *   w_down: hidden x ffn               w_lm: vocab x hidden              */
typedef struct ci_decode_layout {
  uint64_t g_attn, w_qkv, w_o, g_mlp, w_gu, w_down;
  uint64_t layer_stride;
  uint64_t g_final, w_lm;
  uint64_t weight_elems;    /* arena size in BF16 elements                     */
  uint64_t cache_elems;     /* per cache tensor: layers x batch x n_kv x max_ctx x head_dim */
  uint64_t workspace_bytes; /* device workspace decode_step needs              */
  uint64_t attn_part_bytes; /* workspace ci_attention_decode needs             */
} ci_decode_layout_t;

/* Validates cfg and fills the layout.  CI_ERR_INVALID_ARG on a bad config. */
ci_status_t decode_layout(const ci_decode_config_t* cfg, ci_decode_layout_t* out);

typedef struct ci_decode_desc {
  ci_decode_config_t cfg;
  const void* weights;  /* device BF16 arena laid out by decode_layout          */
  void* k_cache;        /* device BF16 [layers][batch][n_kv][max_ctx][head_dim] */
  void* v_cache;        /* same shape                                            */
  const int32_t* pos;   /* HOST int32[batch]: position of the new token, in
                           [0, max_ctx); it attends to positions 0 .. pos     */
  const float* x_in;    /* device FP32 [batch][hidden]                          */
  float* x_out;         /* device FP32 [batch][hidden]                          */
  float* logits;        /* device FP32 [batch][vocab]; may be NULL if vocab 0   */
  void* work;           /* device workspace of layout.workspace_bytes           */
  uint32_t flags;       /* CI_DECODE_KERNEL_TIMES or CI_DECODE_GRAPH (not both) or 0 */
  uint32_t reserved;
} ci_decode_desc_t;

typedef struct ci_decode_result {
  double step_ns;                /* the step's launches, from HIP events       */
  double kernel_ns[CI_DK_COUNT]; /* per kernel kind, summed over layers (only
                                    with CI_DECODE_KERNEL_TIMES, else 0)       */
  uint64_t checksum_bits;        /* bit-pattern sum of logits (x_out if vocab 0) */
  double sum_f64;                /* FP64 sum of the same                       */
  uint64_t t_begin, t_end;       /* device clock around the step               */
} ci_decode_result_t;

/* Run one decode step on `stream` and wait for it.  The step reads x_in and
 * the cache, writes entry pos[b] of every layer's cache, x_out and logits;
 * with unchanged inputs, repeated steps give bit-identical outputs, in every
 * mode (flags).  Step time: first kernel start to last kernel end with
 * CI_DECODE_KERNEL_TIMES, else events recorded around the launches (or the
 * graph launch). */
ci_status_t decode_step(ci_ctx_t* ctx, const ci_decode_desc_t* d, void* stream,
                        ci_decode_result_t* out);

typedef struct ci_decode_cell {
  int resource;
  float intensity;
  uint32_t duty;
  int ncu;
  double step_alone_p50, step_alone_p90;  /* ns, over the reps               */
  double step_col_p50, step_col_p90;
  double kernel_alone_ns[CI_DK_COUNT];    /* medians over the reps           */
  double kernel_col_ns[CI_DK_COUNT];
  double stressor_achieved, stressor_pct_peak;  /* means over the reps        */
  int window_covered, output_equal, timed_out, reps;
  int queue_unresolved;                   /* as in ci_cell_t                 */
} ci_decode_cell_t;

/* measure_sensitivity for the decode step: for every resource rs[i] and
 * intensity xs[j], warm up, then `reps` times run a step alone and one
 * colocated with the stressor (persistent mode, shared or disjoint
 * placement), checking stressor window and output of each colocated step.
 * Reports p50/p90 step times and per-kernel medians (Fig. 5 breakdown). */
ci_status_t measure_decode(ci_ctx_t* ctx, const ci_decode_desc_t* d, const ci_resource_t* rs,
                           const ci_stressor_opts_t* sopts, int nr, const float* xs, int nx,
                           const ci_measure_opts_t* o, void* ws, size_t ws_bytes, void* stream,
                           ci_decode_cell_t* cells);

/* The step's GEMV with its fused prologue and epilogue (device pointers,
 * synchronous on `stream`):
 *   input: v (BF16, batch x k) or, when v is NULL, x (FP32, batch x k)
 *     normalised as ci_rmsnorm_bf16 does with gain g and eps, bit for bit;
 *   PLAIN: out[b][i] = res[b][i] (res may be NULL or alias out) + sum_j
 *     w[i][j] in[b][j];
 *   SILU: rows = 2 ffn (gate rows, then up rows); h[b][j] =
 *     bf16(g / (1 + exp(-g)) * u), g and u rows j and ffn + j, as
 *     ci_silu_mul_bf16 computes them;
 *   ROPE: rows = (n_q + 2 n_kv) * head_dim; the outputs go through
 *     ci_rope_append's arithmetic at host positions pos[b]: rotated queries
 *     to q_out, keys and values to entry pos[b] of k_cache / v_cache.
 * w, v, x, g 16-byte aligned; k a multiple of 8; batch 1..8. */
typedef enum ci_gemv_epilogue { CI_GEMV_PLAIN = 0, CI_GEMV_SILU = 1, CI_GEMV_ROPE = 2 } ci_gemv_epilogue_t;

typedef struct ci_gemv_args {
  const void* w;
  uint32_t rows, k, batch;
  int epilogue;               /* ci_gemv_epilogue_t                            */
  const void* v;              /* BF16 input, or NULL                           */
  const float* x;             /* FP32 input to normalise when v is NULL        */
  const void* g;              /* BF16 gain (k)                                 */
  float eps;
  const float* res;           /* PLAIN                                         */
  float* out;
  void* h;                    /* SILU                                          */
  const int32_t* pos;         /* ROPE: HOST int32[batch], each in [0, max_ctx) */
  uint32_t n_q, n_kv, head_dim, max_ctx;
  float rope_base;
  float* q_out;
  void* k_cache;
  void* v_cache;
} ci_gemv_args_t;

ci_status_t ci_fused_gemv(ci_ctx_t* ctx, const ci_gemv_args_t* a, void* stream);

/* The step's stages as separate kernels (device pointers, synchronous on
 * `stream`): the unfused composition the fused GEMV reproduces, for parity
 * tests and for callers composing their own step.
 *   ci_rmsnorm_bf16: y[r] = bf16(x[r] / sqrt(mean(x[r]^2) + eps) * g),
 *     rows x n, n a multiple of 4.
 *   ci_gemv_bf16_rows: out[b][i] = res[b][i] (res may be NULL or alias out)
 *     + sum_j w[i][j] v[b][j]; w rows x k, v batch x k (batch 1..8), k a
 *     multiple of 8, w and v 16-byte aligned.
 *   ci_rope_append: rotates the query and key heads of qkv (batch x
 *     (n_q + 2 n_kv) x head_dim FP32) at position pos[b] (HOST array), writes
 *     the queries to q_out (batch x n_q x head_dim FP32) and the BF16 keys
 *     and values to entry pos[b] of k_cache / v_cache (one layer:
 *     batch x n_kv x max_ctx x head_dim).
 *   ci_attention_decode: out (batch x n_q*head_dim BF16) = softmax(q K^T /
 *     sqrt(head_dim)) V over positions 0 .. pos[b]; part: device scratch of
 *     layout.attn_part_bytes for this batch, n_q, head_dim and max_ctx.
 *   ci_silu_mul_bf16: h[b][j] = bf16(g / (1 + exp(-g)) * u) with
 *     g = gu[b][j], u = gu[b][ffn + j]. */
ci_status_t ci_rmsnorm_bf16(ci_ctx_t* ctx, const float* x, const uint16_t* g, uint32_t rows,
                            uint32_t n, float eps, uint16_t* y, void* stream);
ci_status_t ci_gemv_bf16_rows(ci_ctx_t* ctx, const uint16_t* w, const uint16_t* v, const float* res,
                              float* out, uint32_t rows, uint32_t k, uint32_t batch, void* stream);
ci_status_t ci_rope_append(ci_ctx_t* ctx, const float* qkv, const int32_t* pos, uint32_t batch,
                           uint32_t n_q, uint32_t n_kv, uint32_t head_dim, uint32_t max_ctx,
                           float rope_base, float* q_out, uint16_t* k_cache, uint16_t* v_cache,
                           void* stream);
ci_status_t ci_attention_decode(ci_ctx_t* ctx, const float* q, const uint16_t* k_cache,
                                const uint16_t* v_cache, const int32_t* pos, uint32_t batch,
                                uint32_t n_q, uint32_t n_kv, uint32_t head_dim, uint32_t max_ctx,
                                void* part, size_t part_bytes, uint16_t* out, void* stream);
ci_status_t ci_silu_mul_bf16(ci_ctx_t* ctx, const float* gu, uint32_t batch, uint32_t ffn,
                             uint16_t* h, void* stream);

/* ci_attention_decode without the `part` workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  It allocates nothing: positions and
 * partial results live in a static device array of 256 +
 * CI_NOALLOC_PART_BYTES bytes that each device holds for the life of the
 * process (its address is fetched once per device in ci_init).  Same
 * arguments, kernels and bit-identical output as ci_attention_decode.
 * CI_ERR_INVALID_ARG when the partial results, batch x n_q x
 * ceil(max_ctx / 64) x (head_dim + 2) x 4 bytes, exceed
 * CI_NOALLOC_PART_BYTES (batch 8, n_q 32, head_dim 128 fits max_ctx up to
 * 8064), and for every argument ci_attention_decode rejects.
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind (nothing in it needs clearing: each call rewrites what it reads);
 * calls that overlap on one GPU, from any context or stream, race. */
#define CI_NOALLOC_PART_BYTES (16ull << 20)
ci_status_t ci_attention_decode_noalloc(ci_ctx_t* ctx, const float* q, const uint16_t* k_cache,
                                        const uint16_t* v_cache, const int32_t* pos, uint32_t batch,
                                        uint32_t n_q, uint32_t n_kv, uint32_t head_dim,
                                        uint32_t max_ctx, uint16_t* out, void* stream);

/* ------------------------------------------------------------- serving */
typedef enum ci_policy_kind {
  CI_POLICY_NAIVE = 0,       /* admit when memory and a slot are free          */
  CI_POLICY_USHER = 1,       /* ... and summed occupancy stays below 1         */
  CI_POLICY_SENSITIVITY = 2  /* ... and every predicted slowdown <= bound      */
} ci_policy_kind_t;

#define CI_NPOINTS 5  /* intensities 0, .25, .5, .75, 1 */

/* Sensitivity profile of one workload kind: what the paper's kernel-level
 * interference estimator consumes (Section 5.1 asks a colocation scheduler
 * to predict each kernel's slowdown from its sensitivity to every shared
 * resource and the pressure its co-runners put on them).
 *   sens[r][p]: the kind's measured slowdown (as a victim) beside stressor r
 *     at intensity point p = 0, .25, .5, .75, 1 (the stressor's CU fraction
 *     or its duty cycle on every CU: the caller picks the axis);
 *   press[r]:   the load the kind itself puts on r when it runs alone, as
 *     the equivalent intensity of stressor r on the same axis (0..1): the
 *     intensity at which the stressor's standalone rate matches the kind's
 *     use of r;
 *   occ:        fraction of the GPU's wave slots it fills (USHER policy).
 * Read/write-aware HBM pricing (optional; all-zero sens_hbm_read = absent):
 * the same HBM byte rate costs a victim more when it includes writes, so a
 * co-runner whose HBM traffic is read-mostly is priced on the victim's curve
 * against the read-only HBM mix instead of the triad's.
 *   sens_hbm_read[p]: slowdown curve against the read-only HBM mix;
 *   press_hbm_read:   this kind's HBM load as that mix's equivalent intensity;
 *   hbm_write_frac:   write share of its compulsory HBM bytes (0..1). */
typedef struct ci_profile {
  int kind;                             /* victim kind this profile covers    */
  float sens[CI_RES_COUNT][CI_NPOINTS]; /* measured slowdown curve per resource */
  float press[CI_RES_COUNT];            /* pressure it exerts (0..1)           */
  float occ;                            /* fraction of wave slots it fills     */
  float sens_hbm_read[CI_NPOINTS];
  float press_hbm_read;
  float hbm_write_frac;
} ci_profile_t;

/* A co-runner counts as read-mostly below this write share of its HBM bytes. */
#define CI_READ_MOSTLY_WRITE_FRAC (1.0f / 6.0f)

/* Predicted slowdown of `victim` beside the co-runners (Section 5.1's
 * estimator, in the reading this library takes): the co-runners' loads add
 * per resource, each resource's factor is max(1, curve at the summed load)
 * with the curve linear between its five points and the load clipped to
 * [0, 1], and the factors multiply (a conservative combination).  HBM load
 * from read-mostly co-runners (hbm_write_frac < CI_READ_MOSTLY_WRITE_FRAC) is
 * summed separately, from their press_hbm_read, and priced on the victim's
 * sens_hbm_read curve when the victim has one; all other HBM load is priced
 * on sens[CI_RES_HBM].  nco == 0 gives 1.  Pure host computation; profiles
 * are caller-owned.  CI_ERR_INVALID_ARG on NULL pointers or nco < 0. */
ci_status_t ci_predict_slowdown(const ci_profile_t* victim, const ci_profile_t* const* corunners,
                                int nco, double* out);

typedef struct ci_request {
  double arrival_s;       /* seconds after the loop starts                   */
  int kind;               /* ci_victim_kind_t                                 */
  int dtype;              /* as in ci_victim_desc_t                           */
  uint64_t m, n, k;       /* sizes as in ci_victim_desc_t                     */
  uint64_t seed;          /* input stream seed (uniform [-1, 1) inputs)       */
  /* Optional caller-owned device buffer (NULL = none) that receives a copy
   * of the request's FP32 output (GEMM m x n, GEMV n, triad n) before its
   * arena memory is released, for checking served results. */
  void* out_copy;
} ci_request_t;

typedef struct ci_policy {
  int kind;               /* ci_policy_kind_t                                 */
  double bound;           /* SENSITIVITY: max predicted slowdown              */
  uint64_t hbm_budget;    /* bytes of device memory the loop may hold         */
  int slots;              /* max requests on the device at once (1..8)        */
  const ci_profile_t* profiles;
  int nprofiles;
  /* Optional (NULL = none): the load of a co-runner present for the whole
   * run, such as the stressor serve_run_background holds (its press, occ
   * and read/write fields are read; kind and sens are not). */
  const ci_profile_t* background;
} ci_policy_t;

typedef struct ci_served {
  double arrival_s, admit_s, end_s;  /* host clock, seconds after start       */
  double service_ns;                 /* device time of the request's kernel   */
  uint64_t checksum_bits;
  double sum_f64;
  int slot;
  int status;                        /* ci_status_t of this request           */
} ci_served_t;

/* Inputs of served requests are drawn on the device from the request's seed:
 * with u(s, i) the uniform [-1, 1) draw i of SplitMix64 stream s (the
 * counter form and mapping of the input generator), a triad reads b = u(seed)
 * and c = u(seed + 1); a GEMM reads A = u(seed) (m x k) and B = u(seed + 1)
 * (n x k), rounded to BF16 for BF16 requests; a GEMV reads W = u(seed)
 * (n x k) and x = u(seed + 1) (k), both rounded to BF16.
 *
 * Continuous-batching colocation loop: the interference-aware scheduler of
 * Section 5.1 (decide per kernel, predict each kernel's slowdown from the
 * co-runners' pressure on every resource, trade a bounded slowdown for
 * utilisation), against memory-only admission and the occupancy rule the
 * paper shows failing (Section 3, Pitfall 1).  Requests (sorted by
 * arrival_s) arrive in real time; each is admitted FIFO (no bypass) when the
 * policy allows (ci_admit), its inputs are generated and its kernel launched
 * on a free slot stream, and it retires when its completion is observed.  The loop owns
 * one device arena of hbm_budget bytes for all request buffers.  out[i]
 * receives request i's record.  Synchronous; returns when all are done. */
ci_status_t serve_run(ci_ctx_t* ctx, const ci_request_t* trace, int n, const ci_policy_t* p,
                      ci_served_t* out);

/* Pure admission decision used by serve_run (Section 5.1: admit a kernel
 * beside others only when the predicted slowdowns stay within a bound),
 * exposed for testing: running_kinds[0..nrun) and cand_kind name profiles
 * in p; cand_bytes / free_bytes are the candidate's footprint and the
 * largest free block of the loop's arena.  *admit = 0 when the candidate
 * does not fit in memory or every slot is busy; otherwise 1 on an idle
 * device (nrun == 0: the rules below bound colocation only); otherwise
 * NAIVE admits, USHER admits when the summed occupancy of all jobs stays
 * below 1 (Section 3, Pitfall 1), and SENSITIVITY admits when
 * ci_predict_slowdown of every job, beside all the others, is <= bound.
 * A background load (p->background) is one more co-runner of every job
 * and adds its occ to the USHER sum; its own slowdown is not bounded (it is
 * not a request), and it does not change the idle-device rule.
 * CI_ERR_INVALID_ARG on a bad policy or a kind without a profile. */
ci_status_t ci_admit(const ci_policy_t* p, const int* running_kinds, int nrun, int cand_kind,
                     uint64_t cand_bytes, uint64_t free_bytes, int* admit);

/* serve_run on a device under constant background load (Section 4.1 holds a
 * stressor's interference constant for a victim's whole lifetime; here it
 * is held for the whole serving run, so that admission decides on a loaded
 * device).  After its own set-up the loop launches stressor `resource` at
 * CU fraction `intensity` with `opts` and the caller-owned workspace ws
 * (ws_bytes >= ci_workspace_size), as stressor_launch does; opts->passes
 * must be 0 (the stressor runs until stopped) and opts->deadline_ms should
 * exceed the run.  Before the stressor starts, each slot stream is checked
 * against the stressor's queue (a probe triad in the arena, alone and
 * beside an idle kernel on the stressor's CUs and queue; a slot slowed by
 * more than 5 % gets a new stream, and if one stays slowed the stressor's
 * queue is replaced once; counted in ci_queue_stats), since two hardware
 * queues can slow each other with nothing else shared; the check is skipped
 * when the arena holds fewer than 12 MiB or ws has no room for the idle
 * kernel.  The trace's clock starts once the stressor is running;
 * requests are served exactly as by serve_run; after the last one retires
 * the stressor is stopped and its report written to *rep (caller-owned).
 * Admission sees the stressor only through p->background.  A stressor that
 * holds, on every CU, the LDS, registers or wave slots a request's
 * work-groups need keeps that request from starting until the stressor's
 * in-kernel deadline (the resource-fit effect of Section 4.2).  Errors as
 * serve_run and stressor_launch; CI_ERR_INVALID_ARG also for NULL opts or
 * rep, or opts->passes != 0; CI_ERR_TIMEOUT when the stressor stopped on
 * its deadline (out and *rep are still written). */
ci_status_t serve_run_background(ci_ctx_t* ctx, const ci_request_t* trace, int n,
                                 const ci_policy_t* p, ci_resource_t resource, float intensity,
                                 const ci_stressor_opts_t* opts, void* ws, size_t ws_bytes,
                                 ci_served_t* out, ci_stressor_report_t* rep);

#ifdef __cplusplus
}
#endif
#endif /* COLOC_H */
