/*
 * ssa.h -- C ABI of the MI355X (gfx950) rigorous complex-interval
 * Schoenhage-Strassen integer multiplication library (libssa.so).
 *
 * The operation is the one stated in the paper's section 2 (Steinke &
 * Sainudiin, CCA 2010): given x in Z_b^n and y in Z_b^m, little-endian digit
 * vectors (value = sum x_i b^i), return z in Z_b^{n+m} with z = x * y.  The
 * product is computed by the fast convolution of section 2.3 over rectangular
 * complex intervals with outward rounding (section 2.5), and each convolution
 * coefficient is taken as the unique integer in its enclosure; when an
 * enclosure holds more than one integer the product is not returned and the
 * status says so (section 1: "report an error").  A returned product is
 * therefore exact (a computer-aided proof of the product), never approximate.
 *
 * Conventions for every entry point
 *  - Operands and results are BYTES (base 256, little-endian).  digit_bits = 4
 *    only changes the internal digit base (each byte is split into two base-16
 *    digits, low nibble first); the interface stays in bytes.
 *  - Pointers named a, b, out, status_dev, and the debug buffers are DEVICE
 *    pointers (hipMalloc'd memory or tensors of the calling framework) owned by
 *    the caller.  Host pointers are named *_host or are plain size arrays.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *  - The library never reads outside [a, a+na), [b, b+nb) and never writes
 *    outside [out, out+na+nb).
 *  - Return value: SSA_OK, or the error that prevented the call from running
 *    (invalid argument, out of memory, device error).  The outcome of a product
 *    (certified or not) is reported separately in its status.
 *  - Thread safety: a plan is used by one host thread at a time.
 */
#ifndef SSA_H_
#define SSA_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SSA_OK = 0,                 /* product certified; out holds the exact na+nb bytes */
  SSA_ENCLOSURE_TOO_WIDE = 1, /* some enclosure held >1 integer; out is all zeros   */
  SSA_INVALID_ARGUMENT = 2,   /* null pointer, zero length, size above the plan's max */
  SSA_OUT_OF_MEMORY = 3,      /* device or pinned host allocation failed             */
  SSA_DEVICE_ERROR = 4,       /* a HIP call failed, or the carry scan gave up         */
  SSA_INTERNAL_ERROR = 5      /* an enclosure excluded every integer: cannot happen
                                 for rigorous arithmetic; out is all zeros           */
} ssa_status;

enum { SSA_FP64 = 0, SSA_FP32_FALLBACK = 1 };
enum { SSA_ARITH_RECT = 0, SSA_ARITH_DISC = 1, SSA_ARITH_NAIVE = 2, SSA_ARITH_NAIVE32 = 3 };
enum { SSA_CERTIFY_ONE_INTEGER = 0, SSA_CERTIFY_HALF_INTEGER = 1 };

typedef struct {
  int precision;           /* SSA_FP64: the path of the paper, all in FP64 intervals.
                              SSA_FP32_FALLBACK: products that the plan's length
                              predictor admits first run their forward
                              transform in FP32 midpoint-radius discs (circular
                              containment sets, section 4; the rest stays FP64);
                              any product that this attempt cannot certify is
                              re-run on the device in FP64.  Same products.     */
  int digit_bits;          /* 8: base-256 digits (paper, section 3); 4: base 16        */
  int certify_mode;        /* SSA_CERTIFY_ONE_INTEGER: exactly one integer (section 1);
                              SSA_CERTIFY_HALF_INTEGER: additionally fail any enclosure
                              that contains a half-integer (stricter)                 */
  int separate_transforms; /* 0 (default): both real operands go through ONE complex
                              interval FFT of a + i b and are separated afterwards
                              (A_k = (Z_k + conj Z_{-k})/2, B_k = (Z_k - conj Z_{-k})/2i);
                              1: one forward FFT per operand, as in the fast
                              convolution box of section 2.3.  Same products.       */
  int refine_digits;       /* 0 (default) or 1 with digit_bits = 8: ssa_mul re-runs a
                              product whose enclosures hold several integers with
                              base-16 digits (coefficients 289 times smaller, a
                              transform twice as long) when that transform is at most
                              2^22 points; the plan allocates for it.  The product is
                              the same; stats.refined says which run produced it.
                              Batches report the base-256 outcome.                 */
  int arithmetic;          /* SSA_ARITH_RECT (default): rectangular complex intervals
                              (section 2.5) everywhere.  SSA_ARITH_DISC: the FP64
                              transforms, products and certification run in
                              midpoint-radius discs (circular containment sets,
                              section 4), which a rotation by a root of unity does not
                              enlarge; the FP32 attempt's forward transform is a disc
                              transform either way.  Needs the packed transform
                              (separate_transforms = 0; SSA_INVALID_ARGUMENT
                              otherwise) and launch shapes without the persistent
                              row pass.  Same products.
                              SSA_ARITH_NAIVE: NOT RIGOROUS, a baseline for the cost
                              of the intervals: the same kernels on plain complex
                              doubles rounded to nearest, each coefficient rounded to
                              the nearest integer without a certificate; the product
                              can be wrong and the status only says the run ended.
                              stats.max_radius holds the largest distance of a
                              coefficient to its integer.  Needs precision SSA_FP64,
                              the packed transform, no refinement, and launch shapes
                              without the persistent row pass.
                              SSA_ARITH_NAIVE32: NOT RIGOROUS, the same in single
                              precision (float complex points, the double twiddles
                              rounded to float): the arithmetic of section 1's remark
                              that a naive single-precision transform is sometimes
                              wrong at 120 base-256 digits.  Only products whose
                              transform fits one workgroup (ssa_fft_size <= 4096);
                              the plan's max_na + max_nb must give such a length.  */
  int refine_disc;         /* 0 (default) or 1 with arithmetic = SSA_ARITH_RECT and the
                              packed transform: ssa_mul re-runs a product whose
                              rectangular enclosures hold several integers once more
                              in FP64 discs (same digits, same length), before any
                              base-16 refinement; stats.refined = 2 when that run
                              produced it.  Batches report the first outcome.     */
  int fp64_digit_bits;     /* 0 (default): every product uses digit_bits.  8, with
                              precision SSA_FP32_FALLBACK and digit_bits = 4: a
                              product that the length predictor does not give to the
                              FP32 attempt goes straight to the FP64 path with base-256
                              digits (a transform half as long as base 16 needs);
                              the FP32 attempt and its re-runs keep base 16.  ssa_mul
                              re-runs a base-256 product refused as too wide with
                              base-16 digits (stats.refined = 1); batches report the
                              base-256 outcome.  Same products.                    */
  int exact_fallback;      /* 0 (default): a product that every interval run refuses
                              is reported as SSA_ENCLOSURE_TOO_WIDE (section 1:
                              report an error).  1: ssa_mul then computes it with
                              the other algorithm section 1 allows: the same fast
                              convolution (section 2.3) by a number-theoretic
                              transform over Z_p, p = 2^64 - 2^32 + 1, exact by
                              construction (the idea of the paper's second,
                              finite-ring Schoenhage-Strassen algorithm), so such a
                              plan's ssa_mul always returns the product
                              (stats.refined = 3).  Products whose interval
                              transform would exceed 2^22 points go to it directly,
                              up to na + nb - 1 <= 2^27 bytes; the plan allocates 56
                              bytes per point of that transform.  Not with
                              SSA_ARITH_NAIVE.  Batches never use it (products
                              beyond 2^22 points are rejected there).            */
} ssa_plan_opts;

typedef struct {
  double max_radius;   /* max over coefficients of the real-part half-width, rounded up */
  uint64_t half_int;   /* coefficients whose enclosure contains a half-integer         */
  uint32_t too_wide;   /* coefficients whose enclosure holds several integers          */
  uint32_t internal;   /* enclosures that exclude every integer (must be 0)            */
  uint32_t carry_err;  /* carry-scan waits that timed out (must be 0)                  */
  uint32_t log_n;      /* transform length used, N = 2^log_n                           */
  int status;          /* ssa_status of the product                                    */
  int fallback;        /* 1: the FP32 attempt failed and the FP64 re-run produced the
                          result (SSA_FP32_FALLBACK plans only)                         */
  int fp32_attempt;    /* 1: the product went through an FP32 attempt                  */
  int refined;         /* 1: base 256 was too wide and the base-16 re-run produced it
                          (plans with refine_digits or fp64_digit_bits); 2: the
                          rectangles were too wide
                          and the re-run in discs produced it (refine_disc); 3: the
                          exact number-theoretic transform produced it
                          (exact_fallback; max_radius is then 0)                */
} ssa_stats;

typedef struct ssa_plan ssa_plan;
typedef struct ssa_batch ssa_batch;

/* Transform length N = 2^k with k = ceil(log2(L)), L = digits(a) + digits(b) - 1
 * (section 2.3, fast convolution box, generalised to unequal lengths); products
 * with L <= 256 are padded to N = 512 (zero padding does not change them). */
size_t ssa_fft_size(size_t na, size_t nb, int digit_bits);

/* Create a plan for products with na <= max_na, nb <= max_nb bytes.  Allocates
 * all device scratch once (ssa_mul never allocates), generates the certified
 * twiddle table on the device (section 2.2 half-angle recurrence) and waits
 * for it.  opts may be NULL (FP64, base 256, one-integer certification).
 * The longest product's transform (ssa_fft_size) must be at most 2^22 points,
 * or with opts->exact_fallback at most 2^27 base-256 points (na, nb <= 2^31);
 * SSA_INVALID_ARGUMENT otherwise.  On error *plan is NULL. */
ssa_status ssa_plan_create(ssa_plan **plan, size_t max_na, size_t max_nb,
                           const ssa_plan_opts *opts, void *stream);

/* Release a plan and everything it allocated (the section 2.2 twiddle table,
 * scratch, pinned staging; no paper passage beyond that: resource handling);
 * waits for the plan's stream first.  Batches created from the plan must be
 * destroyed before it.  NULL is ignored. */
void ssa_plan_destroy(ssa_plan *plan);

/* z = a * b (section 2, long multiplication box: x in Z_b^n, y in Z_b^m ->
 * z in Z_b^{n+m}), computed by the Schoenhage-Strassen box of section 2.4: the
 * fast convolution of section 2.3 over complex intervals (section 2.5), then
 * certification of every coefficient and the carry loop.
 *  - a: na bytes, b: nb bytes, out: na + nb bytes, all device memory owned by
 *    the caller; 1 <= na <= max_na and 1 <= nb <= max_nb of the plan, else
 *    SSA_INVALID_ARGUMENT.  Leading zero bytes and zero operands are allowed.
 *  - *status (host) receives the outcome.  SSA_OK: out holds the exact product
 *    (its top byte may be 0).  SSA_ENCLOSURE_TOO_WIDE: some enclosure held
 *    several integers in every run the plan allows (section 1: report an
 *    error; the refine_* options add runs), out is zero-filled.
 *    SSA_INTERNAL_ERROR: an enclosure excluded every integer, which rigorous
 *    arithmetic cannot produce; out is zero-filled.
 *  - Runs on the plan's stream and synchronises it; allocates nothing. */
ssa_status ssa_mul(ssa_plan *plan, const uint8_t *a, size_t na, const uint8_t *b, size_t nb,
                   uint8_t *out, ssa_status *status);

/* z = a * b by long multiplication (section 2.1, LM box), the O(na nb) method
 * that section 3 times the Schoenhage-Strassen product against: the exact
 * column sums s_i = sum_j a_j b_{i-j} (integer dot products on the GPU), then
 * the LM box's carry loop as the library's carry scan.  Exact, so *status is
 * always SSA_OK.  Same arguments, limits, stream and synchronisation as
 * ssa_mul; uses the plan's scratch (any plan), allocates nothing. */
ssa_status ssa_mul_long(ssa_plan *plan, const uint8_t *a, size_t na, const uint8_t *b, size_t nb,
                        uint8_t *out, ssa_status *status);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the product
 * of ssa_mul for a plan with the default options (FP64 rectangles, base 256,
 * packed transform, one-integer certification), with no plan and no
 * allocation.  The scratch (twiddle table, transform array, coefficients,
 * statistics, carry state, descriptor: about 18.1 MiB) is one static device
 * array per GPU, held until the process ends.
 *  - a: na bytes, b: nb bytes, out: na + nb bytes, status_dev: one int, all
 *    device memory owned by the caller.  na + nb - 1 <= 2^18 (75,000-byte
 *    operands fit; transforms of at most 2^18 points), else
 *    SSA_INVALID_ARGUMENT and nothing is enqueued.
 *  - *status_dev receives the ssa_status of the product (SSA_OK: out holds the
 *    exact product; otherwise out is zero-filled), stream-ordered on `stream`;
 *    nothing is synchronised, so the call can be captured into a graph.
 *  - The first call on a device (the current one) finds that device's array,
 *    builds the twiddle table in it and synchronises `stream` once; it must not
 *    be made under stream capture (SSA_INVALID_ARGUMENT).  Later calls only
 *    enqueue kernels.
 *  - All calls on one GPU share its array, and every call leaves its contents
 *    there: calls that overlap on one GPU (different streams, or different
 *    host threads without ordering) race and give wrong products.  Order them
 *    on one stream. */
ssa_status ssa_mul_noalloc(const uint8_t *a, size_t na, const uint8_t *b, size_t nb, uint8_t *out,
                           int *status_dev, void *stream);

/* FP32 policy of an SSA_FP32_FALLBACK plan (the length predictor): a product
 * tries FP32 first when its coefficient count L = digits(a) + digits(b) - 1 is
 * at most max_coeffs (0 <= max_coeffs <= 4096; 0 disables the attempt) and its
 * transform fits one workgroup (N <= 4096); all others run in FP64 directly.
 * The plan starts with a default that depends on digit_bits.  force_fail = 1
 * widens every FP32 disc so that each attempt fails (a test hook for the
 * re-run).  SSA_INVALID_ARGUMENT for an FP64 plan or a value out of range.
 * Batches created afterwards use the new policy. */
ssa_status ssa_plan_set_fp32_policy(ssa_plan *plan, int max_coeffs, int force_fail);

/* Test hook for the failure path: with on = 1, certification treats every
 * coefficient's enclosure as holding several integers, so products report
 * SSA_ENCLOSURE_TOO_WIDE and zero-filled outputs (the carry scan writes zeros).
 * Affects ssa_mul calls and batches created while it is on; on = 0 restores
 * normal certification.  SSA_INVALID_ARGUMENT for another value. */
ssa_status ssa_plan_force_too_wide(ssa_plan *plan, int on);

/* Test hook for the impossible-enclosure path: with index >= 0, certification
 * of coefficient `index` (in the plan's digits) first lowers that enclosure's
 * upper bound by 1, so that an enclosure of radius < 1/2 no longer holds any
 * integer; such a product reports SSA_INTERNAL_ERROR (stats.internal = 1) with a
 * zero-filled output.  The plan's certify_mode is replaced by the one-integer
 * rule while the hook is on.  index = -1 turns it off; ssa_plan_force_too_wide
 * takes precedence.  Affects ssa_mul calls and batches created while it is on.
 * SSA_INVALID_ARGUMENT for index < -1 or above 2^30. */
ssa_status ssa_plan_corrupt_bound(ssa_plan *plan, long long index);

/* Statistics of the last ssa_mul on this plan (host copy): the largest
 * real-part radius of the coefficient enclosures (the width of section 2.5's
 * intervals, halved and rounded up), the half-integer and failure counts, the
 * transform length and which run produced the result.  No device work. */
ssa_status ssa_get_stats(const ssa_plan *plan, ssa_stats *stats_host);

/* Batches: `count` independent products of uneven lengths, each within the
 * plan's max_na / max_nb, each certified on its own (section 1: detection per
 * instance, so one refused product does not affect the others).  The arrays a, na, b, nb, out are HOST arrays of
 * device pointers and byte counts.  Creation validates every product,
 * allocates the batch's device scratch (the batch owns it), groups the
 * products by transform length, uploads the work descriptors and captures the
 * whole launch sequence into one HIP graph. */
ssa_status ssa_batch_create(ssa_plan *plan, size_t count, const uint8_t *const *a,
                            const size_t *na, const uint8_t *const *b, const size_t *nb,
                            uint8_t *const *out, ssa_batch **batch);
/* Run a batch (one graph launch, stream-ordered, no host synchronisation).
 * status_dev: device array of `count` ints, receives each product's ssa_status
 * (section 1: the certified product, or the error for that product alone). */
ssa_status ssa_batch_run(ssa_batch *batch, int *status_dev);
/* Per-product statistics of the last run (host array of `count`: the section 2.5
 * enclosure radius and the counts of ssa_stats); synchronises. */
ssa_status ssa_batch_stats(ssa_batch *batch, ssa_stats *stats_host);
/* Release a batch and its device scratch and graph (resource handling); NULL is
 * ignored. */
void ssa_batch_destroy(ssa_batch *batch);

/* Run a batch without its graph, with a HIP event recorded on the plan's
 * stream right before and right after every kernel launch (for timing). */
ssa_status ssa_batch_run_timed(ssa_batch *batch, int *status_dev);
/* Kernel time of the timed runs since the previous call, summed per kernel
 * kind into ms_host[6] (milliseconds) with the launch counts in
 * launches_host[6]: 0 single-workgroup product, 1 forward column pass,
 * 2 row pass (forward rows, pointwise product, inverse rows), 3 inverse
 * column pass with scaling and certification, 4 carry scan, 5 status.
 * Synchronises the plan's stream. */
ssa_status ssa_batch_kernel_times(ssa_batch *batch, double *ms_host, int *launches_host);

/* Convenience: create, run, synchronise, destroy.  Each product is certified
 * on its own (section 1's per-instance detection): one product's too-wide
 * enclosure sets only its own status (device array of `count` ints) and
 * zero-fills only its own output.  Allocates the batch's scratch for the call. */
ssa_status ssa_mul_batch(ssa_plan *plan, size_t count, const uint8_t *const *a, const size_t *na,
                         const uint8_t *const *b, const size_t *nb, uint8_t *const *out,
                         int *status_dev);

/* Batched forward interval DFT (section 2.2: X_k = sum_n x_n omega^{n k} with
 * omega = e^{+2 pi i / N}) over rectangular complex intervals with outward
 * rounding (section 2.5), by the same two-pass four-step kernels as a product's
 * forward transform: column DFTs of length N1 times omega_N^{n2 k1}, then row
 * DFTs of length N2 = N / N1.
 *  - log_n: 12 < log_n <= the plan's largest transform length; count: 1..65535.
 *  - x (device, read): count vectors of N = 2^log_n elements in natural order,
 *    each element 4 doubles {re_lo, re_hi, im_lo, im_hi} with lo <= hi.
 *  - y (device, written): count vectors of N elements in four-step order: with
 *    N1 = 2^(*log_n1_host) and N2 = N / N1, element k1 * N2 + k2 of vector v
 *    encloses X_v[k1 + N1 k2].  x and y must not overlap (SSA_INVALID_ARGUMENT).
 *  - The launch shape is the plan's for log_n (ssa_plan_get_config; the row pass
 *    holds 2 * rows rows per workgroup for packed plans, rows otherwise).
 *  - pass_ms_host (nullable, host, 2 doubles): when given, the plan's stream is
 *    synchronised and the column and row pass times (ms, HIP events) stored.
 * Stream-ordered on the plan's stream; allocates nothing when pass_ms_host is NULL. */
ssa_status ssa_fft_forward(ssa_plan *plan, int log_n, size_t count, const double *x, double *y,
                           int *log_n1_host, double *pass_ms_host);

/* ---- Launch shapes and the autotuner ----------------------------------------- */

/* Launch shape of the three-pass path (transforms longer than 2^12) for one
 * transform length 2^log_n: column transforms of length 2^log_n1 (rows of
 * 2^(log_n - log_n1)), `cols` adjacent columns per forward column-pass
 * workgroup, `rows` rows (row pairs for the packed transform) per row-pass
 * workgroup, whether the row pass runs persistent, and `inv_cols` adjacent
 * columns per inverse column-pass workgroup. */
typedef struct {
  int log_n1;
  int cols;
  int rows;
  int persistent;  /* 1: the row pass runs as a persistent kernel (as many workgroups as
                      are resident) that prefetches its next rows while computing the
                      current ones; packed plans with rows of at most 2^9 points only */
  int inv_cols;    /* set_config: 0 means the same as cols; get_config and the
                      autotuner return the value in use */
} ssa_launch_config;

ssa_status ssa_plan_get_config(const ssa_plan *plan, int log_n, ssa_launch_config *cfg_host);
/* Rejects (SSA_INVALID_ARGUMENT) shapes that do not fit the kernels: workgroups
 * over 512 threads or not whole wavefronts, LDS over 64 KiB, uneven grids. */
ssa_status ssa_plan_set_config(ssa_plan *plan, int log_n, const ssa_launch_config *cfg_host);
/* Times every valid shape with inv_cols == cols for transforms of length
 * 2^log_n (12 < log_n <= the plan's largest) on `count` synthetic products of
 * that length in the digits such products run in (fp64_digit_bits when the
 * plan sets it, else digit_bits; SSA_INVALID_ARGUMENT when the plan's operand
 * limits allow no product of that length) (device memory allocated for the
 * call and released), then, from
 * the fastest, every other inv_cols and after that every other cols; keeps the
 * fastest in the plan and returns it with its time per batch of `count`
 * products (milliseconds) and the number of shapes tried.  Synchronises the
 * plan's stream. */
ssa_status ssa_plan_autotune(ssa_plan *plan, int log_n, int count, ssa_launch_config *best_host,
                             double *best_ms_host, int *tried_host);

/* ---- Diagnostics used by the test-suite ------------------------------------ */

/* Same computation as ssa_mul, and also writes the final enclosures of all N
 * convolution outputs (after the inverse transform and the 1/N factor, before
 * certification) to enc_dev: N x 4 doubles {re_lo, re_hi, im_lo, im_hi}, with N
 * the transform length of the plan's own digit size (no base-16 refinement).
 * Lengths above 2^12 run the half-length inverse of the real coefficients, whose
 * enclosures are real: there im_lo = im_hi = 0. */
ssa_status ssa_debug_enclosures(ssa_plan *plan, const uint8_t *a, size_t na, const uint8_t *b,
                                size_t nb, uint8_t *out, double *enc_dev, ssa_status *status);

/* Copy the plan's twiddle table: Ntab x 2 doubles (cos, sin of 2 pi t / Ntab)
 * to tab_dev, and its common error bound to *e_host.  Returns log2(Ntab) in
 * *log_ntab_host.  Ntab is the longest transform the plan allocates for: that of
 * max_na x max_nb in its digit size, or the base-16 one with refine_digits. */
ssa_status ssa_twiddle_table(const ssa_plan *plan, double *tab_dev, double *e_host,
                             int *log_ntab_host);

/* The device directed-rounding primitives on n inputs (device arrays):
 * op 0 RU(a+b), 1 RU(a*b), 2 RU(a*b+c), 3 RD(a+b), 4 RD(a*b), 5 RD(a*b+c).
 * Synchronises the stream. */
ssa_status ssa_probe_directed(int op, const double *a, const double *b, const double *c,
                              double *out, size_t n, void *stream);

/* The device certification step (section 1: the unique integer in each
 * enclosure, else an error) on caller-supplied enclosures, for testing it
 * against the CPU oracle.
 *  - enc_dev (device, read): n x 4 doubles {re_lo, re_hi, im_lo, im_hi},
 *    1 <= n <= 2^31.  Entries i < L are coefficient enclosures; entries
 *    L <= i < n are padded-tail enclosures, which must contain 0 in both parts.
 *  - mode: SSA_CERTIFY_ONE_INTEGER or SSA_CERTIFY_HALF_INTEGER.
 *  - c_dev (device, written, may be NULL when L = 0): L int64 coefficients, 0
 *    where an entry is not certified.
 *  - cls_dev (device, written, nullable): n ints, the entry's outcome: 0 one
 *    integer, 1 several integers (too wide), 5 impossible (no integer, a single
 *    negative one or one of 2^52 and more, an imaginary part or a tail entry
 *    excluding 0), plus 16 when the real part contains a half-integer.
 *  - stats_host (host, written): status (SSA_INTERNAL_ERROR over
 *    SSA_ENCLOSURE_TOO_WIDE over SSA_OK), max_radius (largest RU((re_hi -
 *    re_lo)/2) over i < L), half_int, too_wide and internal counts.
 * Allocates a few bytes of device memory for the call and synchronises the
 * stream (NULL = default).  SSA_INVALID_ARGUMENT for bad sizes or mode. */
ssa_status ssa_probe_certify(const double *enc_dev, size_t n, size_t L, int mode, int64_t *c_dev,
                             int *cls_dev, ssa_stats *stats_host, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SSA_H_ */
