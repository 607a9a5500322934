// Shared declarations between the kernels and the C-ABI implementation.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "ia.hpp"

namespace ssa {

// Per-product statistics, accumulated on the device.
struct dev_stats {
  unsigned long long max_rad_bits;  // bit pattern of max real-part radius (>= 0)
  unsigned long long half_int;      // enclosures containing a half-integer
  unsigned int too_wide;            // enclosures holding more than one integer
  unsigned int internal;            // enclosures that cannot be rigorous
  unsigned int carry_err;           // carry scan gave up waiting (never expected)
  unsigned int fallback;            // 1: the FP32 attempt failed, the FP64 re-run ran
  unsigned int fp32;                // 1: an FP32 attempt was made
};

enum { HOOK_FORCE_FP32_FAIL = 1 };

// One product as the kernels see it.  Sizes are in digits of the chosen base.
struct task {
  const uint8_t *a;
  const uint8_t *b;
  uint8_t *out;
  uint32_t na, nb;        // operand bytes
  uint32_t nda, ndb;      // operand digits (bytes, or nibbles when digit_bits == 4)
  uint32_t L;             // coefficient count nda + ndb - 1
  uint32_t log_n;         // transform length N = 2^log_n
  ci *ya;                 // multi-pass scratch: N elements per operand
  ci *yb;
  unsigned long long *c;  // coefficients (N entries)
  dev_stats *st;
  uint32_t *tiles;        // carry-scan tile status words
  uint32_t ntiles;
  uint32_t fp32;          // 1: FP32 first attempt, FP64 re-run on failure
};

// Element types of the transforms (the values of ssa_plan_opts.arithmetic);
// single-precision points only in the single-workgroup kernel.
enum { ARITH_RECT = 0, ARITH_DISC = 1, ARITH_POINT = 2, ARITH_POINT32 = 3 };

// CERT_FORCE_TOO_WIDE: test hook, every coefficient counts as too wide.
// Modes from CERT_CORRUPT_BASE on: test hook, one-integer certification with
// the upper bound of coefficient (mode - CERT_CORRUPT_BASE) lowered by 1
// before it is certified (an enclosure that no longer holds its integer).
enum { CERT_ONE_INTEGER = 0, CERT_HALF_INTEGER = 1, CERT_FORCE_TOO_WIDE = 2, CERT_CORRUPT_BASE = 4 };

// Tile of the carry scan: 4 wavefronts x 8 chunks of 64 positions (half the LDS of 16 chunks, so twice the resident tiles: 15% faster).
static constexpr int CARRY_THREADS = 256;
static constexpr int CARRY_CHUNKS = 8;
static constexpr int CARRY_TILE = CARRY_THREADS * CARRY_CHUNKS;
// Tile status words sit one 128-byte line apart, so that spinning readers of
// one tile do not contend with the publication of its neighbours.
static constexpr uint32_t TILE_WORD_STRIDE = 32;

// Largest transform done by one workgroup holding everything in LDS, and the
// smallest transform length (shorter products are zero-padded to it).
static constexpr int SMALL_MAX_LOG = 12;
static constexpr int SMALL_MIN_LOG = 9;

struct launch_cfg {
  int log_n1;  // column transform length (multi-pass)
  int log_n2;  // row transform length
  int cols;    // columns per workgroup in the column passes
  int rows;    // rows (row pairs when packed) per workgroup in the row pass
  int pack;    // 1: one complex transform of a + i b; 0: one transform per operand
  int persist; // 1: persistent row-pair pass with next-item prefetch (pack, rows <= 2^9)
  int icols;   // columns per workgroup in the inverse column pass
  int arith;   // element type: ARITH_RECT, ARITH_DISC or ARITH_POINT (the last two: packed,
               // plain row pass)
};

// Default launch shape of the three-pass path for N = 2^log_n.
launch_cfg default_launch_cfg(int log_n, int pack, int arith);
// Raises every product kernel's dynamic-LDS limit (once per process).
hipError_t set_kernel_attributes();

struct twtab_host {
  const double2 *tab;
  int log_ntab;
  double e;
};

// Optional timing: mark(ctx, kind, 0) right before and mark(ctx, kind, 1) right
// after each kernel launch, on the launch stream.
enum {
  KIND_SMALL = 0,
  KIND_COL_FWD = 1,
  KIND_ROW = 2,
  KIND_COL_INV = 3,
  KIND_CARRY = 4,
  KIND_STATUS = 5,
  KIND_COUNT = 6
};
struct timing_hook {
  void (*mark)(void *ctx, int kind, int phase);
  void *ctx;
};

// dbg (nullable): N x 4 doubles {re_lo, re_hi, im_lo, im_hi} of the final
// enclosures of task 0, written before certification.
// fp32: FP32 first attempt over tasks that are all marked fp32; rerun: FP64
// pass that follows it, skipping marked tasks that the attempt certified.
hipError_t launch_small(const task *d_tasks, int ntasks, int log_n, int digit_bits, int cert_mode,
                        int pack, int arith, int fp32, int rerun, int hooks, const twtab_host &tw,
                        double *dbg, hipStream_t s, const timing_hook *hk = nullptr);
hipError_t launch_multipass(const task *d_tasks, int ntasks, int log_n, const launch_cfg &cfg,
                            int digit_bits, int cert_mode, const twtab_host &tw, double *dbg,
                            hipStream_t s, const timing_hook *hk = nullptr);
// Batched forward DFT of `count` vectors of N = N1 N2 public-layout intervals
// (x -> y, four-step output order); ev (nullable): 3 events recorded before the
// column pass, between the passes and after the row pass.
hipError_t launch_fft_forward(const double *x, double *y, int count, const launch_cfg &cfg,
                              const twtab_host &tw, hipStream_t s, hipEvent_t *ev);
hipError_t launch_carry(const task *d_tasks, int ntasks, uint32_t max_tiles, int digit_bits,
                        hipStream_t s, const timing_hook *hk = nullptr);
// Carries over an explicit list of (task index, tile) pairs, one workgroup each
// (ntiles >= 1 entries in d_map; every product's tiles consecutive, ascending).
hipError_t launch_carry_map(const task *d_tasks, const uint2 *d_map, uint32_t ntiles,
                            int digit_bits, hipStream_t s, const timing_hook *hk = nullptr);
hipError_t launch_status(const task *d_tasks, int ntasks, int *d_status, hipStream_t s,
                         const timing_hook *hk = nullptr);
hipError_t launch_directed_probe(int op, const double *a, const double *b, const double *c,
                                 double *out, size_t n, hipStream_t s);
// Certification of n caller-supplied enclosures (n x 4 doubles {re_lo, re_hi,
// im_lo, im_hi}) of which the first L are coefficients: coefficients to c
// (L entries), per-entry outcome to cls (nullable), totals accumulated into
// *st (zeroed by the caller).
hipError_t launch_certify_probe(const double *enc, uint32_t n, uint32_t L, int mode,
                                unsigned long long *c, int *cls, dev_stats *st, hipStream_t s);

// The exact transform (ntt.hip): roots of unity of Z_p, p = 2^64 - 2^32 + 1, by
// level (lv[2^l + u] = w_{2^l}^u, 2^(K+1) entries, wK of order 2^K), and one
// product's convolution coefficients into task.c (task.ya: 4 N residues of
// scratch); the carry scan follows separately.
hipError_t make_ntt_levels(int K, uint64_t wK, uint64_t *lv, hipStream_t s);
// Long multiplication (lm.hip): the column sums of task d_task into its
// coefficients (zeroed first, with the statistics and carry state).
hipError_t launch_long_mul(const task *d_task, const task &h_task, hipStream_t s);
hipError_t launch_ntt_product(const task *d_task, const task &h_task, int log_n, const uint64_t *lv,
                              uint64_t ninv, hipStream_t s);

}  // namespace ssa
