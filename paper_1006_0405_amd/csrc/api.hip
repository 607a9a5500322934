// C ABI (include/ssa.h): plans, single products, batches, diagnostics.
//
// A plan owns the certified twiddle table for its largest transform, the
// scratch of one product and pinned staging for its descriptor and
// statistics; ssa_mul only enqueues kernels and one small copy each way.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "../../include/ssa.h"
#include "internal.hpp"
#include "twiddle.hpp"

using namespace ssa;

namespace {

constexpr int MAX_LOG_N = 22;  // N1 = N2 = 2^11: 1024-thread column and 512-thread row passes
// Longest exact (number-theoretic) transform: base-256 operands of up to
// 2^26 bytes each; every coefficient stays below 2^26 255^2 < 2^42.
constexpr int MAX_NTT_LOG = 27;
constexpr uint64_t NTT_P = 0xFFFFFFFF00000001ull;  // 2^64 - 2^32 + 1

uint64_t host_mulmod(uint64_t a, uint64_t b) {
  return static_cast<uint64_t>(static_cast<unsigned __int128>(a) * b % NTT_P);
}
uint64_t host_powmod(uint64_t w, uint64_t e) {
  uint64_t r = 1;
  for (; e; e >>= 1, w = host_mulmod(w, w))
    if (e & 1) r = host_mulmod(r, w);
  return r;
}
// A root of unity of order exactly 2^K in Z_p: 7^((p - 1) / 2^32) has order
// 2^32 (its 2^31-th power is -1), and its 2^(32 - K)-th power has order 2^K.
// Returns 0 if that check fails.
uint64_t ntt_root(int K) {
  const uint64_t w32 = host_powmod(7, (NTT_P - 1) >> 32);
  if (host_powmod(w32, uint64_t(1) << 31) != NTT_P - 1) return 0;
  const uint64_t w = host_powmod(w32, uint64_t(1) << (32 - K));
  if (K > 0 && host_powmod(w, uint64_t(1) << (K - 1)) != NTT_P - 1) return 0;
  return w;
}

int ceil_log2(uint64_t v) {
  int k = 0;
  while ((uint64_t(1) << k) < v) ++k;
  return k;
}

// Transform length exponent for L coefficients (zero padding up to 2^SMALL_MIN_LOG = 2^9).
int log_n_for(uint64_t L) { return std::max(ceil_log2(L), SMALL_MIN_LOG); }

uint64_t digits(size_t n, int bits) { return bits == 4 ? 2 * uint64_t(n) : uint64_t(n); }

// Default launch shape of the three-pass path for N = 2^log_n (8 elements per
// thread): C adjacent columns per column-pass workgroup (256 threads, 512 for
// N1 = 2^11), and G rows (or row pairs) per row-pass workgroup.
static_assert(ARITH_RECT == SSA_ARITH_RECT && ARITH_DISC == SSA_ARITH_DISC &&
                  ARITH_POINT == SSA_ARITH_NAIVE && ARITH_POINT32 == SSA_ARITH_NAIVE32,
              "the kernels' element types follow ssa_plan_opts.arithmetic");

}  // namespace

launch_cfg ssa::default_launch_cfg(int log_n, int pack, int arith) {
  launch_cfg c;
  c.log_n1 = log_n / 2;
  c.log_n2 = log_n - c.log_n1;
  const int N1 = 1 << c.log_n1, N2 = 1 << c.log_n2;
  c.cols = std::max(2, std::min(32, 2048 / N1));
  c.pack = pack;
  c.persist = 0;
  c.icols = c.cols;
  c.arith = arith;
  const int t = N2 / 8;  // threads per row
  if (pack)
    c.rows = std::max(1, std::min(N1 / 2, 128 / t));
  else
    c.rows = std::max(1, std::min(N1, 256 / t));
  return c;
}

namespace {

// A launch shape is usable when every workgroup has at most 512 threads in
// whole wavefronts, its LDS (exchange buffers with one spare slot per 8
// elements) fits in 80 KiB, and the grids divide evenly.
bool cfg_valid(const launch_cfg &c, int log_n) {
  if (c.log_n1 < 6 || c.log_n1 > 11 || log_n - c.log_n1 < 6 || log_n - c.log_n1 > 11) return false;
  if (c.log_n2 != log_n - c.log_n1) return false;
  const int N1 = 1 << c.log_n1, N2 = 1 << c.log_n2;
  const auto pow2 = [](int x) { return x > 0 && (x & (x - 1)) == 0; };
  const auto cols_ok = [&](int cols, int ncols) {
    const int ct = cols * N1 / 8;
    return pow2(cols) && ncols % cols == 0 && ct <= 512 && ct % 64 == 0 &&
           (N1 + N1 / 8) * static_cast<size_t>(cols) * 16 <= 81920;
  };
  if (!cols_ok(c.cols, N2) || !cols_ok(c.icols, N2 / 2)) return false;  // inverse: N2/2 columns
  const int per = c.pack ? 2 : 1;
  if (!pow2(c.rows) || (c.pack ? (N1 / 2) % c.rows : N1 % c.rows)) return false;
  const int rt = per * c.rows * N2 / 8;
  if (rt > 512 || rt % 64) return false;
  if (static_cast<size_t>(per) * c.rows * (N2 + N2 / 8) * 16 > 81920) return false;
  if (c.persist != 0 && c.persist != 1) return false;
  // discs and points: packed transform, plain row pass
  if (c.arith != ARITH_RECT && (!c.pack || c.persist)) return false;
  // the persistent row pass: packed rows of one wavefront, twiddle levels in LDS
  if (c.persist && (!c.pack || c.log_n2 > 9 ||
                    (2 * static_cast<size_t>(c.rows) * (N2 + N2 / 8) + (size_t(2) << c.log_n2)) * 16 > 81920))
    return false;
  return true;
}

bool hip_ok(hipError_t e) { return e == hipSuccess; }

// Default length predictor of the FP32 first attempt: the largest coefficient
// count L for which random and all-0xFF operands still certify.  Radii add
// linearly through the butterflies while magnitudes grow like a square root,
// and the pointwise product multiplies a forward radius by the other
// operand's transform, so the coefficient radius grows like n^1.5 U b^2 and
// doubles with each extra radix-2 level: base-256 digits leave room only for
// products of a few bytes, base 16 certifies while the transform has 512
// points (L <= 511) and mostly fails from 1024 points on.
constexpr uint32_t FP32_MAX_L_B256 = 7, FP32_MAX_L_B16 = 511;
uint32_t default_fp32_max_L(int digit_bits) { return digit_bits == 8 ? FP32_MAX_L_B256 : FP32_MAX_L_B16; }

int status_from(const dev_stats &s) {
  if (s.internal) return SSA_INTERNAL_ERROR;
  if (s.too_wide) return SSA_ENCLOSURE_TOO_WIDE;
  if (s.carry_err) return SSA_DEVICE_ERROR;
  return SSA_OK;
}

ssa_stats to_public(const dev_stats &s, int log_n) {
  ssa_stats o;
  std::memset(&o, 0, sizeof(o));
  uint64_t rb = s.max_rad_bits;
  std::memcpy(&o.max_radius, &rb, sizeof(double));
  o.half_int = s.half_int;
  o.too_wide = s.too_wide;
  o.internal = s.internal;
  o.carry_err = s.carry_err;
  o.log_n = static_cast<uint32_t>(log_n);
  o.status = status_from(s);
  o.fallback = static_cast<int>(s.fallback);
  o.fp32_attempt = static_cast<int>(s.fp32);
  o.refined = 0;
  return o;
}

bool kernels_configured = false;

// Concurrent branches of a batch graph: each multi-pass class is split into
// this many parts, one per stream, each part followed by its own carry scan.
// Two measured fastest: 64 products of 75,000 bytes take 0.414 ms per graph
// launch with two branches, 0.439 ms with four (and 0.434 ms with two branches
// whose carries waited for both).
constexpr int GRAPH_BRANCHES = 2;
static_assert(GRAPH_BRANCHES >= 1 && GRAPH_BRANCHES <= 8, "graph branches: 1..8 streams");

// Part of a class of n products (slots s0 .. s0 + n) that slot k belongs to when
// the class is split into `parts` (part q: slots s0 + q n / parts onwards).
int part_of(size_t k, size_t s0, size_t n, int parts) {
  const size_t off = k - s0;
  int q = 0;
  while (q + 1 < parts && off >= (q + 1) * n / parts) ++q;
  return q;
}

}  // namespace

struct ssa_plan {
  int device = 0;
  hipStream_t stream = nullptr;
  ssa_plan_opts opts{};
  uint32_t fp32_max_L = 0;  // FP32 first attempt for products with L <= this (0: never)
  int hooks = 0;         // test hooks (HOOK_FORCE_FP32_FAIL)
  int force_too_wide = 0;  // test hook: certification refuses every coefficient
  int corrupt_index = -1;  // test hook: coefficient whose upper bound is lowered by 1 (-1: off)
  int split_graph = GRAPH_BRANCHES;  // batch graphs run each multi-pass class as this many
                                     // concurrent parts (1: one stream)
  size_t max_na = 0, max_nb = 0;
  int log_nmax = 0;
  int log_nref = 0;  // refine_digits: largest base-16 re-run transform (0: none)
  int log_nntt = 0;  // exact_fallback: longest exact transform (0: none)
  uint64_t *ntt_lv = nullptr;  // exact_fallback: roots of unity of Z_p by level
  // twiddles
  double2 *tab = nullptr;
  int log_ntab = 0;
  double e = 0.0;
  unsigned long long *ebits = nullptr;
  void *roots = nullptr;
  // single-product scratch
  ci *ya = nullptr, *yb = nullptr;
  unsigned long long *c = nullptr;
  dev_stats *st = nullptr;
  uint32_t *tiles = nullptr;
  task *d_task = nullptr;
  task *h_task = nullptr;       // pinned
  dev_stats *h_stats = nullptr; // pinned
  ssa_stats last{};
  launch_cfg cfg[MAX_LOG_N + 1];  // multi-pass launch shape per transform length
};

struct ssa_batch {
  ssa_plan *plan = nullptr;
  size_t count = 0;
  std::vector<int> order;  // task slot -> caller index
  task *d_tasks = nullptr;
  std::vector<task> h_tasks;
  std::vector<int> bits;  // digit size by task slot
  ci *arena = nullptr;
  unsigned long long *carena = nullptr;
  dev_stats *stats = nullptr;
  uint32_t *tiles = nullptr;
  int *d_status_slot = nullptr;  // by slot
  int *d_status = nullptr;       // by caller index
  int *d_order = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint32_t max_tiles = 0;
  size_t n_multi = 0;
  uint2 *d_tile_map = nullptr;  // (task slot, tile) per carry workgroup
  uint32_t total_tiles = 0;
  // the same tiles grouped by graph branch (graph form: each branch's carries
  // run on its own stream), branch 0's products first
  uint2 *d_tile_map_split = nullptr;
  uint32_t branch_tiles[8] = {};
  // timed (eager) runs: one event before and one after every kernel launch
  std::vector<hipEvent_t> events;
  std::vector<int> kinds;
  size_t ev_used = 0;
  bool ev_error = false;
};

namespace {

void free_plan(ssa_plan *p) {
  if (!p) return;
  (void)hipFree(p->tab);
  (void)hipFree(p->ebits);
  (void)hipFree(p->roots);
  (void)hipFree(p->ntt_lv);
  (void)hipFree(p->ya);
  (void)hipFree(p->yb);
  (void)hipFree(p->c);
  (void)hipFree(p->st);
  (void)hipFree(p->tiles);
  (void)hipFree(p->d_task);
  if (p->h_task) (void)hipHostFree(p->h_task);
  if (p->h_stats) (void)hipHostFree(p->h_stats);
  delete p;
}

twtab_host tw_of(const ssa_plan *p) { return twtab_host{p->tab, p->log_ntab, p->e}; }

// The FP32 twiddle bound assumes a table error below 2^-47 (it always is, by
// many orders of magnitude).
bool fp32_first(const ssa_plan *p, uint64_t L, int log_n) {
  return p->opts.precision == SSA_FP32_FALLBACK && log_n <= SMALL_MAX_LOG &&
         L <= p->fp32_max_L && p->e < 0x1p-47;
}

// Digit size of a product's first run: the plan's, unless the plan sends the
// products that the FP32 attempt is not given to FP64 with other digits.
int route_bits(const ssa_plan *p, size_t na, size_t nb) {
  const int bits = p->opts.digit_bits;
  if (p->opts.fp64_digit_bits == 0) return bits;
  const uint64_t L = digits(na, bits) + digits(nb, bits) - 1;
  return fp32_first(p, L, log_n_for(L)) ? bits : p->opts.fp64_digit_bits;
}

// Enqueue one product class: all tasks [d_tasks, d_tasks + n) share log_n, and
// the first n32 of them are marked for the FP32 first attempt.
hipError_t enqueue_class(const ssa_plan *p, const task *d_tasks, int n, int n32, int log_n,
                         double *dbg, hipStream_t s, const timing_hook *hk = nullptr,
                         int bits = 0) {
  if (bits == 0) bits = p->opts.digit_bits;
  const int mode = p->force_too_wide        ? CERT_FORCE_TOO_WIDE
                   : p->corrupt_index >= 0 ? CERT_CORRUPT_BASE + p->corrupt_index
                                           : p->opts.certify_mode;
  const int pack = p->opts.separate_transforms ? 0 : 1;
  const int arith = p->opts.arithmetic;
  if (log_n <= SMALL_MAX_LOG) {
    if (n32 == 0)
      return launch_small(d_tasks, n, log_n, bits, mode, pack, arith, 0, 0, 0, tw_of(p), dbg, s, hk);
    // FP32 attempt, then FP64 over the class except what the attempt certified
    const hipError_t e = launch_small(d_tasks, n32, log_n, bits, mode, pack, arith, 1, 0, p->hooks,
                                      tw_of(p), dbg, s, hk);
    if (e != hipSuccess) return e;
    return launch_small(d_tasks, n, log_n, bits, mode, pack, arith, 0, 1, 0, tw_of(p), dbg, s, hk);
  }
  // the multi-pass kernels index products by a grid dimension (at most 65535)
  constexpr int MAX_GRID_PRODUCTS = 65535;
  for (int k0 = 0; k0 < n; k0 += MAX_GRID_PRODUCTS) {
    const hipError_t e = launch_multipass(d_tasks + k0, std::min(MAX_GRID_PRODUCTS, n - k0), log_n,
                                          p->cfg[log_n], bits, mode, tw_of(p), dbg, s, hk);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// One product with the given digit size; the FP32 attempt only in the plan's own.
ssa_status run_once(ssa_plan *p, const uint8_t *a, size_t na, const uint8_t *b, size_t nb,
                    uint8_t *out, double *dbg, ssa_status *status, int bits) {
  const uint64_t nda = digits(na, bits), ndb = digits(nb, bits);
  const uint64_t L = nda + ndb - 1;
  const int log_n = log_n_for(L);
  task &t = *p->h_task;
  std::memset(&t, 0, sizeof(t));
  t.a = a;
  t.b = b;
  t.out = out;
  t.na = static_cast<uint32_t>(na);
  t.nb = static_cast<uint32_t>(nb);
  t.nda = static_cast<uint32_t>(nda);
  t.ndb = static_cast<uint32_t>(ndb);
  t.L = static_cast<uint32_t>(L);
  t.log_n = static_cast<uint32_t>(log_n);
  t.ya = p->ya;
  t.yb = p->yb;
  t.c = p->c;
  t.st = p->st;
  t.tiles = p->tiles;
  t.ntiles = static_cast<uint32_t>((na + nb + CARRY_TILE - 1) / CARRY_TILE);
  t.fp32 = (bits == p->opts.digit_bits && fp32_first(p, L, log_n)) ? 1u : 0u;
  hipStream_t s = p->stream;
  if (!hip_ok(hipMemcpyAsync(p->d_task, p->h_task, sizeof(task), hipMemcpyHostToDevice, s)))
    return SSA_DEVICE_ERROR;
  if (!hip_ok(enqueue_class(p, p->d_task, 1, static_cast<int>(t.fp32), log_n, dbg, s, nullptr,
                            bits)))
    return SSA_DEVICE_ERROR;
  if (log_n > SMALL_MAX_LOG && !hip_ok(launch_carry(p->d_task, 1, t.ntiles, bits, s)))
    return SSA_DEVICE_ERROR;
  if (!hip_ok(hipMemcpyAsync(p->h_stats, p->st, sizeof(dev_stats), hipMemcpyDeviceToHost, s)))
    return SSA_DEVICE_ERROR;
  if (!hip_ok(hipStreamSynchronize(s))) return SSA_DEVICE_ERROR;
  p->last = to_public(*p->h_stats, log_n);
  *status = static_cast<ssa_status>(p->last.status);
  return SSA_OK;
}

// The exact last resort: the product by a number-theoretic transform over
// Z_p with base-256 digits, then the same carry scan.  Always certified.
ssa_status run_ntt(ssa_plan *p, const uint8_t *a, size_t na, const uint8_t *b, size_t nb,
                   uint8_t *out, ssa_status *status) {
  const uint64_t L = uint64_t(na) + nb - 1;
  const int log_n = log_n_for(L);
  if (log_n > p->log_nntt) return SSA_INVALID_ARGUMENT;
  task &t = *p->h_task;
  std::memset(&t, 0, sizeof(t));
  t.a = a;
  t.b = b;
  t.out = out;
  t.na = t.nda = static_cast<uint32_t>(na);
  t.nb = t.ndb = static_cast<uint32_t>(nb);
  t.L = static_cast<uint32_t>(L);
  t.log_n = static_cast<uint32_t>(log_n);
  t.ya = p->ya;
  t.c = p->c;
  t.st = p->st;
  t.tiles = p->tiles;
  t.ntiles = static_cast<uint32_t>((na + nb + CARRY_TILE - 1) / CARRY_TILE);
  const uint64_t ninv = host_powmod(uint64_t(1) << log_n, NTT_P - 2);
  hipStream_t s = p->stream;
  if (!hip_ok(hipMemcpyAsync(p->d_task, p->h_task, sizeof(task), hipMemcpyHostToDevice, s)) ||
      !hip_ok(launch_ntt_product(p->d_task, t, log_n, p->ntt_lv, ninv, s)) ||
      !hip_ok(launch_carry(p->d_task, 1, t.ntiles, 8, s)) ||
      !hip_ok(hipMemcpyAsync(p->h_stats, p->st, sizeof(dev_stats), hipMemcpyDeviceToHost, s)) ||
      !hip_ok(hipStreamSynchronize(s)))
    return SSA_DEVICE_ERROR;
  p->last = to_public(*p->h_stats, log_n);
  p->last.refined = 3;
  *status = static_cast<ssa_status>(p->last.status);
  return SSA_OK;
}

ssa_status run_single(ssa_plan *p, const uint8_t *a, size_t na, const uint8_t *b, size_t nb,
                      uint8_t *out, double *dbg, ssa_status *status) {
  if (!p || !a || !b || !out || !status || na == 0 || nb == 0 || na > p->max_na ||
      nb > p->max_nb)
    return SSA_INVALID_ARGUMENT;
  const int bits0 = dbg ? p->opts.digit_bits : route_bits(p, na, nb);
  // products longer than the interval kernels reach go straight to the exact
  // transform (plans with exact_fallback only: others never admit them)
  if (log_n_for(digits(na, bits0) + digits(nb, bits0) - 1) > p->log_nmax) {
    if (dbg || !p->opts.exact_fallback) return SSA_INVALID_ARGUMENT;
    return run_ntt(p, a, na, b, nb, out, status);
  }
  ssa_status r = run_once(p, a, na, b, nb, out, dbg, status, bits0);
  // refinement in discs: the same transform once more with circular enclosures
  if (r == SSA_OK && *status == SSA_ENCLOSURE_TOO_WIDE && p->opts.refine_disc && !dbg) {
    const int log_n = static_cast<int>(p->last.log_n);
    const launch_cfg keep = p->cfg[log_n];
    if (log_n > SMALL_MAX_LOG) {  // a disc launch shape: the plain row pass
      p->cfg[log_n].arith = ARITH_DISC;
      p->cfg[log_n].persist = 0;
    }
    p->opts.arithmetic = SSA_ARITH_DISC;
    r = run_once(p, a, na, b, nb, out, dbg, status, bits0);
    p->opts.arithmetic = SSA_ARITH_RECT;
    p->cfg[log_n] = keep;
    p->last.refined = 2;
  }
  // refinement: a base-256 product whose enclosures are too wide, again in base 16
  // (not for ssa_debug_enclosures: its buffer holds the base-256 transform only)
  if (r == SSA_OK && *status == SSA_ENCLOSURE_TOO_WIDE && p->opts.refine_digits && !dbg &&
      log_n_for(digits(na, 4) + digits(nb, 4) - 1) <= p->log_nref) {
    r = run_once(p, a, na, b, nb, out, dbg, status, 4);
    p->last.refined = 1;
  }
  // a base-256 first run of a base-16 plan (fp64_digit_bits): again in the plan's digits
  if (r == SSA_OK && *status == SSA_ENCLOSURE_TOO_WIDE && bits0 != p->opts.digit_bits) {
    r = run_once(p, a, na, b, nb, out, dbg, status, p->opts.digit_bits);
    p->last.refined = 1;
  }
  // every interval run refused: the exact transform (section 1: another algorithm)
  if (r == SSA_OK && *status == SSA_ENCLOSURE_TOO_WIDE && p->opts.exact_fallback && !dbg)
    r = run_ntt(p, a, na, b, nb, out, status);
  return r;
}

}  // namespace

extern "C" {

size_t ssa_fft_size(size_t na, size_t nb, int digit_bits) {
  if (na == 0 || nb == 0 || (digit_bits != 8 && digit_bits != 4)) return 0;
  return size_t(1) << log_n_for(digits(na, digit_bits) + digits(nb, digit_bits) - 1);
}

ssa_status ssa_plan_create(ssa_plan **plan, size_t max_na, size_t max_nb,
                           const ssa_plan_opts *opts, void *stream) {
  if (!plan) return SSA_INVALID_ARGUMENT;
  *plan = nullptr;
  ssa_plan_opts o{SSA_FP64, 8, SSA_CERTIFY_ONE_INTEGER, 0};  // packed transform
  if (opts) o = *opts;
  if (max_na == 0 || max_nb == 0 || (o.digit_bits != 8 && o.digit_bits != 4) ||
      (o.certify_mode != SSA_CERTIFY_ONE_INTEGER && o.certify_mode != SSA_CERTIFY_HALF_INTEGER) ||
      (o.precision != SSA_FP64 && o.precision != SSA_FP32_FALLBACK) ||
      (o.separate_transforms != 0 && o.separate_transforms != 1) ||
      (o.refine_digits != 0 && (o.refine_digits != 1 || o.digit_bits != 8)) ||
      (o.arithmetic != SSA_ARITH_RECT && o.arithmetic != SSA_ARITH_DISC &&
       o.arithmetic != SSA_ARITH_NAIVE && o.arithmetic != SSA_ARITH_NAIVE32) ||
      (o.arithmetic != SSA_ARITH_RECT && o.separate_transforms != 0) ||
      ((o.arithmetic == SSA_ARITH_NAIVE || o.arithmetic == SSA_ARITH_NAIVE32) &&
       (o.precision != SSA_FP64 || o.refine_digits != 0)) ||
      (o.refine_disc != 0 && (o.refine_disc != 1 || o.arithmetic != SSA_ARITH_RECT ||
                              o.separate_transforms != 0)) ||
      (o.fp64_digit_bits != 0 && (o.fp64_digit_bits != 8 || o.digit_bits != 4 ||
                                  o.precision != SSA_FP32_FALLBACK)) ||
      (o.exact_fallback != 0 &&
       (o.exact_fallback != 1 || o.arithmetic == SSA_ARITH_NAIVE || o.arithmetic == SSA_ARITH_NAIVE32)))
    return SSA_INVALID_ARGUMENT;
  const uint64_t L = digits(max_na, o.digit_bits) + digits(max_nb, o.digit_bits) - 1;
  // the exact transform takes base-256 digits
  const int log_nntt = o.exact_fallback ? log_n_for(uint64_t(max_na) + max_nb - 1) : 0;
  if (log_nntt > MAX_NTT_LOG || max_na > (size_t(1) << 31) || max_nb > (size_t(1) << 31))
    return SSA_INVALID_ARGUMENT;
  // longer products than the interval kernels reach: only with the exact transform
  if (log_n_for(L) > MAX_LOG_N && !o.exact_fallback) return SSA_INVALID_ARGUMENT;
  // single precision points: the single-workgroup kernel only
  if (o.arithmetic == SSA_ARITH_NAIVE32 && log_n_for(L) > SMALL_MAX_LOG) return SSA_INVALID_ARGUMENT;
  const int log_nmax = std::min(log_n_for(L), MAX_LOG_N);
  // the base-16 re-run of refine_digits, as far as a transform of 2^MAX_LOG_N reaches
  const int log_nref =
      o.refine_digits ? std::min(log_n_for(digits(max_na, 4) + digits(max_nb, 4) - 1), MAX_LOG_N) : 0;
  const int log_nalloc = std::max(log_nmax, log_nref);
  if (!kernels_configured) {
    if (!hip_ok(set_kernel_attributes())) return SSA_DEVICE_ERROR;
    kernels_configured = true;
  }
  ssa_plan *p = new (std::nothrow) ssa_plan();
  if (!p) return SSA_OUT_OF_MEMORY;
  p->stream = static_cast<hipStream_t>(stream);
  (void)hipGetDevice(&p->device);
  p->opts = o;
  if (o.precision == SSA_FP32_FALLBACK) p->fp32_max_L = default_fp32_max_L(o.digit_bits);
  p->max_na = max_na;
  p->max_nb = max_nb;
  p->log_nmax = log_nmax;
  p->log_nref = log_nref;
  p->log_nntt = log_nntt;
  p->log_ntab = log_nalloc;
  for (int l = SMALL_MAX_LOG + 1; l <= MAX_LOG_N; ++l)
    p->cfg[l] = default_launch_cfg(l, o.separate_transforms ? 0 : 1, o.arithmetic);
  const size_t N = size_t(1) << log_nalloc;
  const size_t Nntt = log_nntt ? size_t(1) << log_nntt : 0;
  const size_t ntiles = (max_na + max_nb + CARRY_TILE - 1) / CARRY_TILE;
  // transform array: N interval elements (32 bytes) or four arrays of Nntt
  // residues (the same 32 bytes per point)
  const size_t ya_elems = std::max(log_nalloc > SMALL_MAX_LOG ? N : 0, Nntt);
  static_assert(sizeof(ci) == 4 * sizeof(uint64_t), "an exact product uses four residue arrays");
  bool ok = hip_ok(hipMalloc(&p->tab, sizeof(double2) << (p->log_ntab + 1))) &&  // level tables
            hip_ok(hipMalloc(&p->ebits, sizeof(unsigned long long))) &&
            hip_ok(hipMalloc(&p->roots, twiddle_roots_bytes())) &&
            hip_ok(hipMalloc(&p->c, sizeof(unsigned long long) * std::max(N, Nntt))) &&
            hip_ok(hipMalloc(&p->st, sizeof(dev_stats))) &&
            hip_ok(hipMalloc(&p->tiles, sizeof(uint32_t) * TILE_WORD_STRIDE * ntiles)) &&
            hip_ok(hipMalloc(&p->d_task, sizeof(task))) &&
            hip_ok(hipHostMalloc(&p->h_task, sizeof(task), hipHostMallocDefault)) &&
            hip_ok(hipHostMalloc(&p->h_stats, sizeof(dev_stats), hipHostMallocDefault));
  if (ok && ya_elems)
    ok = hip_ok(hipMalloc(&p->ya, sizeof(ci) * ya_elems));  // the packed transform needs one array
  if (ok && log_nalloc > SMALL_MAX_LOG && o.separate_transforms)
    ok = hip_ok(hipMalloc(&p->yb, sizeof(ci) * N));
  if (ok && log_nntt)
    ok = hip_ok(hipMalloc(&p->ntt_lv, sizeof(uint64_t) * 2 * Nntt));
  if (!ok) {
    free_plan(p);
    (void)hipGetLastError();
    return SSA_OUT_OF_MEMORY;
  }
  // certified twiddles: the bound e is read back once and passed by value
  unsigned long long eb = 0;
  ok = hip_ok(hipMemcpyAsync(p->ebits, &eb, sizeof(eb), hipMemcpyHostToDevice, p->stream)) &&
       hip_ok(make_twiddles(p->log_ntab, p->tab + N, p->ebits, p->roots, p->stream)) &&
       hip_ok(make_level_tables(p->log_ntab, p->tab, p->stream)) &&
       (!log_nntt || (ntt_root(log_nntt) != 0 &&
                      hip_ok(make_ntt_levels(log_nntt, ntt_root(log_nntt), p->ntt_lv, p->stream)))) &&
       hip_ok(hipMemcpyAsync(&eb, p->ebits, sizeof(eb), hipMemcpyDeviceToHost, p->stream)) &&
       hip_ok(hipStreamSynchronize(p->stream));
  if (!ok) {
    free_plan(p);
    return SSA_DEVICE_ERROR;
  }
  std::memcpy(&p->e, &eb, sizeof(double));
  *plan = p;
  return SSA_OK;
}

void ssa_plan_destroy(ssa_plan *plan) {
  if (!plan) return;
  (void)hipStreamSynchronize(plan->stream);
  free_plan(plan);
}

ssa_status ssa_mul(ssa_plan *plan, const uint8_t *a, size_t na, const uint8_t *b, size_t nb,
                   uint8_t *out, ssa_status *status) {
  return run_single(plan, a, na, b, nb, out, nullptr, status);
}

ssa_status ssa_mul_long(ssa_plan *plan, const uint8_t *a, size_t na, const uint8_t *b, size_t nb,
                        uint8_t *out, ssa_status *status) {
  ssa_plan *p = plan;
  if (!p || !a || !b || !out || !status || na == 0 || nb == 0 || na > p->max_na || nb > p->max_nb)
    return SSA_INVALID_ARGUMENT;
  const uint64_t L = uint64_t(na) + nb - 1;
  task &t = *p->h_task;
  std::memset(&t, 0, sizeof(t));
  t.a = a;
  t.b = b;
  t.out = out;
  t.na = t.nda = static_cast<uint32_t>(na);
  t.nb = t.ndb = static_cast<uint32_t>(nb);
  t.L = static_cast<uint32_t>(L);
  t.log_n = static_cast<uint32_t>(log_n_for(L));
  t.c = p->c;
  t.st = p->st;
  t.tiles = p->tiles;
  t.ntiles = static_cast<uint32_t>((na + nb + CARRY_TILE - 1) / CARRY_TILE);
  hipStream_t s = p->stream;
  if (!hip_ok(hipMemcpyAsync(p->d_task, p->h_task, sizeof(task), hipMemcpyHostToDevice, s)) ||
      !hip_ok(launch_long_mul(p->d_task, t, s)) ||
      !hip_ok(launch_carry(p->d_task, 1, t.ntiles, 8, s)) ||
      !hip_ok(hipMemcpyAsync(p->h_stats, p->st, sizeof(dev_stats), hipMemcpyDeviceToHost, s)) ||
      !hip_ok(hipStreamSynchronize(s)))
    return SSA_DEVICE_ERROR;
  p->last = to_public(*p->h_stats, 0);
  *status = static_cast<ssa_status>(p->last.status);
  return SSA_OK;
}

ssa_status ssa_debug_enclosures(ssa_plan *plan, const uint8_t *a, size_t na, const uint8_t *b,
                                size_t nb, uint8_t *out, double *enc_dev, ssa_status *status) {
  if (!enc_dev) return SSA_INVALID_ARGUMENT;
  return run_single(plan, a, na, b, nb, out, enc_dev, status);
}

ssa_status ssa_fft_forward(ssa_plan *plan, int log_n, size_t count, const double *x, double *y,
                           int *log_n1_host, double *pass_ms_host) {
  if (!plan || !x || !y || !log_n1_host || log_n <= SMALL_MAX_LOG || log_n > plan->log_nmax ||
      count == 0 || count > 65535)
    return SSA_INVALID_ARGUMENT;
  const size_t bytes = (sizeof(ci) * count) << log_n;
  const char *xb = reinterpret_cast<const char *>(x), *yb = reinterpret_cast<const char *>(y);
  if (xb < yb + bytes && yb < xb + bytes) return SSA_INVALID_ARGUMENT;  // overlap
  launch_cfg c = plan->cfg[log_n];
  if (c.pack) c.rows *= 2;  // the row-pair kernel's workgroup holds 2 rows per pair
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  if (pass_ms_host) {
    for (hipEvent_t &e : ev)
      if (!hip_ok(hipEventCreate(&e))) {
        for (hipEvent_t f : ev)
          if (f) (void)hipEventDestroy(f);
        return SSA_DEVICE_ERROR;
      }
  }
  hipStream_t s = plan->stream;
  bool ok = hip_ok(launch_fft_forward(x, y, static_cast<int>(count), c, tw_of(plan), s,
                                      pass_ms_host ? ev : nullptr));
  if (ok && pass_ms_host) {
    float m0 = 0.f, m1 = 0.f;
    ok = hip_ok(hipEventSynchronize(ev[2])) && hip_ok(hipEventElapsedTime(&m0, ev[0], ev[1])) &&
         hip_ok(hipEventElapsedTime(&m1, ev[1], ev[2]));
    pass_ms_host[0] = m0;
    pass_ms_host[1] = m1;
  }
  for (hipEvent_t f : ev)
    if (f) (void)hipEventDestroy(f);
  if (!ok) return SSA_DEVICE_ERROR;
  *log_n1_host = c.log_n1;
  return SSA_OK;
}

ssa_status ssa_plan_set_fp32_policy(ssa_plan *plan, int max_coeffs, int force_fail) {
  if (!plan || plan->opts.precision != SSA_FP32_FALLBACK || max_coeffs < 0 ||
      max_coeffs > (1 << SMALL_MAX_LOG) || (force_fail != 0 && force_fail != 1))
    return SSA_INVALID_ARGUMENT;
  plan->fp32_max_L = static_cast<uint32_t>(max_coeffs);
  plan->hooks = force_fail ? HOOK_FORCE_FP32_FAIL : 0;
  return SSA_OK;
}

ssa_status ssa_plan_force_too_wide(ssa_plan *plan, int on) {
  if (!plan || (on != 0 && on != 1)) return SSA_INVALID_ARGUMENT;
  plan->force_too_wide = on;
  return SSA_OK;
}

ssa_status ssa_plan_corrupt_bound(ssa_plan *plan, long long index) {
  if (!plan || index < -1 || index > (1ll << 30)) return SSA_INVALID_ARGUMENT;
  plan->corrupt_index = static_cast<int>(index);
  return SSA_OK;
}

ssa_status ssa_get_stats(const ssa_plan *plan, ssa_stats *stats_host) {
  if (!plan || !stats_host) return SSA_INVALID_ARGUMENT;
  *stats_host = plan->last;
  return SSA_OK;
}

ssa_status ssa_twiddle_table(const ssa_plan *plan, double *tab_dev, double *e_host,
                             int *log_ntab_host) {
  if (!plan || !tab_dev || !e_host || !log_ntab_host) return SSA_INVALID_ARGUMENT;
  if (!hip_ok(hipMemcpyAsync(tab_dev, plan->tab + (size_t(1) << plan->log_ntab),
                             sizeof(double2) << plan->log_ntab,
                             hipMemcpyDeviceToDevice, plan->stream)) ||
      !hip_ok(hipStreamSynchronize(plan->stream)))
    return SSA_DEVICE_ERROR;
  *e_host = plan->e;
  *log_ntab_host = plan->log_ntab;
  return SSA_OK;
}

ssa_status ssa_probe_certify(const double *enc_dev, size_t n, size_t L, int mode, int64_t *c_dev,
                             int *cls_dev, ssa_stats *stats_host, void *stream) {
  if (!enc_dev || !stats_host || n == 0 || n > (size_t(1) << 31) || L > n || (L > 0 && !c_dev) ||
      (mode != SSA_CERTIFY_ONE_INTEGER && mode != SSA_CERTIFY_HALF_INTEGER))
    return SSA_INVALID_ARGUMENT;
  hipStream_t s = static_cast<hipStream_t>(stream);
  dev_stats *st = nullptr;
  if (!hip_ok(hipMalloc(&st, sizeof(dev_stats)))) {
    (void)hipGetLastError();
    return SSA_OUT_OF_MEMORY;
  }
  dev_stats h{};
  const bool ok =
      hip_ok(hipMemsetAsync(st, 0, sizeof(dev_stats), s)) &&
      hip_ok(launch_certify_probe(enc_dev, static_cast<uint32_t>(n), static_cast<uint32_t>(L), mode,
                                  reinterpret_cast<unsigned long long *>(c_dev), cls_dev, st, s)) &&
      hip_ok(hipMemcpyAsync(&h, st, sizeof(dev_stats), hipMemcpyDeviceToHost, s)) &&
      hip_ok(hipStreamSynchronize(s));
  (void)hipFree(st);
  if (!ok) return SSA_DEVICE_ERROR;
  *stats_host = to_public(h, 0);
  return SSA_OK;
}

ssa_status ssa_probe_directed(int op, const double *a, const double *b, const double *c,
                              double *out, size_t n, void *stream) {
  if (!a || !b || !c || !out || op < 0 || op > 5) return SSA_INVALID_ARGUMENT;
  if (n == 0) return SSA_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!hip_ok(launch_directed_probe(op, a, b, c, out, n, s)) || !hip_ok(hipStreamSynchronize(s)))
    return SSA_DEVICE_ERROR;
  return SSA_OK;
}

// ---------------------------------------------------------------------------
// Batches

void ssa_batch_destroy(ssa_batch *bt) {
  if (!bt) return;
  (void)hipFree(bt->d_tile_map_split);
  if (bt->plan) (void)hipStreamSynchronize(bt->plan->stream);
  for (hipEvent_t ev : bt->events) (void)hipEventDestroy(ev);
  if (bt->exec) (void)hipGraphExecDestroy(bt->exec);
  if (bt->graph) (void)hipGraphDestroy(bt->graph);
  (void)hipFree(bt->d_tasks);
  (void)hipFree(bt->arena);
  (void)hipFree(bt->carena);
  (void)hipFree(bt->stats);
  (void)hipFree(bt->tiles);
  (void)hipFree(bt->d_tile_map);
  (void)hipFree(bt->d_status_slot);
  (void)hipFree(bt->d_status);
  (void)hipFree(bt->d_order);
  delete bt;
}

}  // extern "C"

namespace ssa {
// Scatter statuses from task order back to caller order.
hipError_t launch_scatter_status(const int *slot_status, const int *order, int n, int *out,
                                 hipStream_t s);
}

namespace {

// Per length class one launch (or three), then one carry scan over every
// multi-pass product, then the statuses.
// side (graph capture only): nside more streams; each multi-pass class is then
// split into up to nside + 1 parts, part q launched on stream q (stream 0 is
// s) between a fork and a join event, so that the parts' kernels can share the
// GPU (one part's memory phases and latency-bound carries overlap another's
// arithmetic); each stream ends with the carry scan of its own products.
hipError_t enqueue_batch(ssa_batch *bt, hipStream_t s, const timing_hook *hk,
                         hipStream_t *side = nullptr, int nside = 0, hipEvent_t fork = nullptr,
                         hipEvent_t *join = nullptr) {
  const ssa_plan *p = bt->plan;
  size_t s0 = 0;
  const size_t count = bt->count;
  const bool split = side != nullptr && nside > 0 && bt->n_multi >= 2;
  const int branches = split ? nside + 1 : 1;
  const auto stream_of = [&](int q) { return q == 0 ? s : side[q - 1]; };
  if (split) {
    hipError_t e = hipEventRecord(fork, s);
    for (int q = 0; q < nside && e == hipSuccess; ++q) e = hipStreamWaitEvent(side[q], fork, 0);
    if (e != hipSuccess) return e;
  }
  while (s0 < count) {
    size_t s1 = s0;
    const int l = static_cast<int>(bt->h_tasks[s0].log_n), cb = bt->bits[s0];
    while (s1 < count && static_cast<int>(bt->h_tasks[s1].log_n) == l && bt->bits[s1] == cb) ++s1;
    const int n = static_cast<int>(s1 - s0);
    int n32 = 0;
    while (n32 < n && bt->h_tasks[s0 + n32].fp32) ++n32;  // marked tasks lead their class
    if (split && l > SMALL_MAX_LOG && n >= 2) {
      const int parts = std::min(branches, n);
      for (int q = 0; q < parts; ++q) {
        const int b0 = static_cast<int>(size_t(q) * n / parts);
        const int b1 = static_cast<int>(size_t(q + 1) * n / parts);
        const hipError_t e =
            enqueue_class(p, bt->d_tasks + s0 + b0, b1 - b0, 0, l, nullptr, stream_of(q), hk, cb);
        if (e != hipSuccess) return e;
      }
    } else {
      const hipError_t e = enqueue_class(p, bt->d_tasks + s0, n, n32, l, nullptr, s, hk, cb);
      if (e != hipSuccess) return e;
    }
    s0 = s1;
  }
  // one digit size for every multi-pass product (the FP32 attempt is single-workgroup)
  if (split) {
    hipError_t e = hipSuccess;
    uint32_t off = 0;
    for (int q = 0; q < branches && e == hipSuccess; ++q) {
      if (bt->branch_tiles[q])
        e = launch_carry_map(bt->d_tasks, bt->d_tile_map_split + off, bt->branch_tiles[q],
                             bt->bits[0], stream_of(q), hk);
      off += bt->branch_tiles[q];
    }
    for (int q = 0; q < nside && e == hipSuccess; ++q) {
      e = hipEventRecord(join[q], side[q]);
      if (e == hipSuccess) e = hipStreamWaitEvent(s, join[q], 0);
    }
    if (e != hipSuccess) return e;
  } else if (bt->n_multi) {
    hipError_t e = launch_carry_map(bt->d_tasks, bt->d_tile_map, bt->total_tiles, bt->bits[0], s, hk);
    if (e != hipSuccess) return e;
  }
  hipError_t e = launch_status(bt->d_tasks, static_cast<int>(count), bt->d_status_slot, s, hk);
  if (e != hipSuccess) return e;
  return launch_scatter_status(bt->d_status_slot, bt->d_order, static_cast<int>(count),
                               bt->d_status, s);
}

void mark_event(void *ctx, int kind, int phase) {
  ssa_batch *bt = static_cast<ssa_batch *>(ctx);
  if (bt->ev_used == bt->events.size()) {
    hipEvent_t ev = nullptr;
    if (hipEventCreate(&ev) != hipSuccess) {
      bt->ev_error = true;
      return;
    }
    bt->events.push_back(ev);
  }
  if (phase == 0) bt->kinds.push_back(kind);
  if (hipEventRecord(bt->events[bt->ev_used++], bt->plan->stream) != hipSuccess) bt->ev_error = true;
}

}  // namespace

extern "C" {

ssa_status ssa_batch_create(ssa_plan *plan, size_t count, const uint8_t *const *a,
                            const size_t *na, const uint8_t *const *b, const size_t *nb,
                            uint8_t *const *out, ssa_batch **batch) {
  if (!batch) return SSA_INVALID_ARGUMENT;
  *batch = nullptr;
  if (!plan || count == 0 || !a || !na || !b || !nb || !out || count > (1u << 24))
    return SSA_INVALID_ARGUMENT;
  std::vector<int> lg(count), bits(count);
  std::vector<char> f32(count);
  for (size_t i = 0; i < count; ++i) {
    if (!a[i] || !b[i] || !out[i] || na[i] == 0 || nb[i] == 0 || na[i] > plan->max_na ||
        nb[i] > plan->max_nb)
      return SSA_INVALID_ARGUMENT;
    bits[i] = route_bits(plan, na[i], nb[i]);
    const uint64_t L = digits(na[i], bits[i]) + digits(nb[i], bits[i]) - 1;
    lg[i] = log_n_for(L);
    if (lg[i] > plan->log_nmax) return SSA_INVALID_ARGUMENT;  // exact transform: ssa_mul only
    f32[i] = (bits[i] == plan->opts.digit_bits && fp32_first(plan, L, lg[i])) ? 1 : 0;
  }
  ssa_batch *bt = new (std::nothrow) ssa_batch();
  if (!bt) return SSA_OUT_OF_MEMORY;
  bt->plan = plan;
  bt->count = count;
  // group by transform length, largest first, then by digit size; within a
  // group, the products marked for the FP32 attempt first
  bt->order.resize(count);
  for (size_t i = 0; i < count; ++i) bt->order[i] = static_cast<int>(i);
  std::stable_sort(bt->order.begin(), bt->order.end(), [&](int x, int y) {
    if (lg[x] != lg[y]) return lg[x] > lg[y];
    if (bits[x] != bits[y]) return bits[x] > bits[y];
    return f32[x] > f32[y];
  });
  // scratch sizes
  size_t arena_elems = 0, c_elems = 0, tiles = 0;
  for (size_t i = 0; i < count; ++i) {
    const size_t N = size_t(1) << lg[i];
    if (lg[i] > SMALL_MAX_LOG) {
      arena_elems += (plan->opts.separate_transforms ? 2 : 1) * N;  // packed: one array
      c_elems += N;
      tiles += (na[i] + nb[i] + CARRY_TILE - 1) / CARRY_TILE;
    }
  }
  bool ok = hip_ok(hipMalloc(&bt->d_tasks, sizeof(task) * count)) &&
            hip_ok(hipMalloc(&bt->stats, sizeof(dev_stats) * count)) &&
            hip_ok(hipMalloc(&bt->d_status_slot, sizeof(int) * count)) &&
            hip_ok(hipMalloc(&bt->d_status, sizeof(int) * count)) &&
            hip_ok(hipMalloc(&bt->d_order, sizeof(int) * count));
  if (ok && arena_elems)
    ok = hip_ok(hipMalloc(&bt->arena, sizeof(ci) * arena_elems)) &&
         hip_ok(hipMalloc(&bt->carena, sizeof(unsigned long long) * c_elems)) &&
         hip_ok(hipMalloc(&bt->tiles, sizeof(uint32_t) * TILE_WORD_STRIDE * std::max<size_t>(tiles, 1)));
  if (!ok) {
    ssa_batch_destroy(bt);
    (void)hipGetLastError();
    return SSA_OUT_OF_MEMORY;
  }
  bt->h_tasks.resize(count);
  bt->bits.resize(count);
  size_t ao = 0, co = 0, to = 0;
  for (size_t s = 0; s < count; ++s) {
    const int i = bt->order[s];
    bt->bits[s] = bits[i];
    task &t = bt->h_tasks[s];
    std::memset(&t, 0, sizeof(t));
    t.a = a[i];
    t.b = b[i];
    t.out = out[i];
    t.na = static_cast<uint32_t>(na[i]);
    t.nb = static_cast<uint32_t>(nb[i]);
    t.nda = static_cast<uint32_t>(digits(na[i], bits[i]));
    t.ndb = static_cast<uint32_t>(digits(nb[i], bits[i]));
    t.L = t.nda + t.ndb - 1;
    t.log_n = static_cast<uint32_t>(lg[i]);
    t.fp32 = static_cast<uint32_t>(f32[i]);
    t.st = bt->stats + s;
    if (lg[i] > SMALL_MAX_LOG) {
      const size_t N = size_t(1) << lg[i];
      t.ya = bt->arena + ao;
      t.yb = plan->opts.separate_transforms ? bt->arena + ao + N : nullptr;
      ao += (plan->opts.separate_transforms ? 2 : 1) * N;
      t.c = bt->carena + co;
      co += N;
      t.ntiles = static_cast<uint32_t>((na[i] + nb[i] + CARRY_TILE - 1) / CARRY_TILE);
      t.tiles = bt->tiles + to * TILE_WORD_STRIDE;
      to += t.ntiles;
    }
  }
  hipStream_t st = plan->stream;
  ok = hip_ok(hipMemcpyAsync(bt->d_tasks, bt->h_tasks.data(), sizeof(task) * count,
                             hipMemcpyHostToDevice, st)) &&
       hip_ok(hipMemcpyAsync(bt->d_order, bt->order.data(), sizeof(int) * count,
                             hipMemcpyHostToDevice, st)) &&
       hip_ok(hipStreamSynchronize(st));
  if (!ok) {
    ssa_batch_destroy(bt);
    return SSA_DEVICE_ERROR;
  }
  for (size_t k = 0; k < count; ++k)
    if (bt->h_tasks[k].log_n > static_cast<uint32_t>(SMALL_MAX_LOG)) {
      bt->n_multi = k + 1;  // multi-pass classes come first
      bt->max_tiles = std::max(bt->max_tiles, bt->h_tasks[k].ntiles);
      if (bt->bits[k] != bt->bits[0]) {  // the carry launch takes one digit size
        ssa_batch_destroy(bt);
        return SSA_INTERNAL_ERROR;
      }
    }
  // Carry workgroups: the multi-pass products' tiles, products in the reverse of
  // their pass order (the last written is still in cache), tiles ascending.
  if (bt->n_multi) {
    std::vector<uint2> map;
    for (size_t k = bt->n_multi; k-- > 0;)
      for (uint32_t t = 0; t < bt->h_tasks[k].ntiles; ++t) map.push_back(make_uint2(static_cast<uint32_t>(k), t));
    bt->total_tiles = static_cast<uint32_t>(map.size());
    // the parts of every multi-pass class as the graph splits them (a class of
    // n >= 2 products into min(branches, n) parts), so that each branch's
    // carries cover its own products
    const int branches = plan->split_graph;
    std::vector<int> branch(bt->n_multi, 0);
    for (size_t s0 = 0; s0 < bt->n_multi;) {
      size_t s1 = s0;
      while (s1 < bt->n_multi && bt->h_tasks[s1].log_n == bt->h_tasks[s0].log_n &&
             bt->bits[s1] == bt->bits[s0])
        ++s1;
      const size_t n = s1 - s0;
      if (branches > 1 && n >= 2)
        for (size_t k = s0; k < s1; ++k)
          branch[k] = part_of(k, s0, n, std::min<int>(branches, static_cast<int>(n)));
      s0 = s1;
    }
    std::vector<uint2> split_map;
    for (int q = 0; q < branches; ++q)
      for (size_t k = bt->n_multi; k-- > 0;)
        if (branch[k] == q) {
          for (uint32_t t = 0; t < bt->h_tasks[k].ntiles; ++t)
            split_map.push_back(make_uint2(static_cast<uint32_t>(k), t));
          bt->branch_tiles[q] += bt->h_tasks[k].ntiles;
        }
    ok = !map.empty() && split_map.size() == map.size() &&
         hip_ok(hipMalloc(&bt->d_tile_map, sizeof(uint2) * map.size())) &&
         hip_ok(hipMalloc(&bt->d_tile_map_split, sizeof(uint2) * map.size())) &&
         hip_ok(hipMemcpyAsync(bt->d_tile_map, map.data(), sizeof(uint2) * map.size(),
                               hipMemcpyHostToDevice, st)) &&
         hip_ok(hipMemcpyAsync(bt->d_tile_map_split, split_map.data(), sizeof(uint2) * map.size(),
                               hipMemcpyHostToDevice, st)) &&
         hip_ok(hipStreamSynchronize(st));
    if (!ok) {
      ssa_batch_destroy(bt);
      (void)hipGetLastError();
      return SSA_OUT_OF_MEMORY;
    }
  }
  // Capture the launch sequence into one graph.
  const int nside = plan->split_graph - 1;
  hipStream_t cs = nullptr, side[7] = {};
  hipEvent_t fork = nullptr, join[7] = {};
  ok = hip_ok(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) &&
       hip_ok(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
  for (int q = 0; q < nside && ok; ++q)
    ok = hip_ok(hipStreamCreateWithFlags(&side[q], hipStreamNonBlocking)) &&
         hip_ok(hipEventCreateWithFlags(&join[q], hipEventDisableTiming));
  if (ok) ok = hip_ok(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  if (ok) ok = hip_ok(enqueue_batch(bt, cs, nullptr, nside > 0 ? side : nullptr, nside, fork, join));
  hipGraph_t g = nullptr;
  if (cs) {
    const hipError_t ec = hipStreamEndCapture(cs, &g);
    ok = ok && hip_ok(ec);
  }
  if (ok) {
    bt->graph = g;
    ok = hip_ok(hipGraphInstantiate(&bt->exec, g, nullptr, nullptr, 0));
  } else if (g) {
    (void)hipGraphDestroy(g);
  }
  if (cs) (void)hipStreamDestroy(cs);
  for (int q = 0; q < nside; ++q) {
    if (side[q]) (void)hipStreamDestroy(side[q]);
    if (join[q]) (void)hipEventDestroy(join[q]);
  }
  if (fork) (void)hipEventDestroy(fork);
  if (!ok) {
    ssa_batch_destroy(bt);
    (void)hipGetLastError();
    return SSA_DEVICE_ERROR;
  }
  *batch = bt;
  return SSA_OK;
}

ssa_status ssa_batch_run(ssa_batch *bt, int *status_dev) {
  if (!bt || !status_dev) return SSA_INVALID_ARGUMENT;
  hipStream_t s = bt->plan->stream;
  if (!hip_ok(hipGraphLaunch(bt->exec, s))) return SSA_DEVICE_ERROR;
  if (!hip_ok(hipMemcpyAsync(status_dev, bt->d_status, sizeof(int) * bt->count,
                             hipMemcpyDeviceToDevice, s)))
    return SSA_DEVICE_ERROR;
  return SSA_OK;
}

ssa_status ssa_batch_run_timed(ssa_batch *bt, int *status_dev) {
  if (!bt || !status_dev) return SSA_INVALID_ARGUMENT;
  hipStream_t s = bt->plan->stream;
  timing_hook hk{mark_event, bt};
  if (!hip_ok(enqueue_batch(bt, s, &hk)) || bt->ev_error) return SSA_DEVICE_ERROR;
  if (!hip_ok(hipMemcpyAsync(status_dev, bt->d_status, sizeof(int) * bt->count,
                             hipMemcpyDeviceToDevice, s)))
    return SSA_DEVICE_ERROR;
  return SSA_OK;
}

ssa_status ssa_batch_kernel_times(ssa_batch *bt, double *ms_host, int *launches_host) {
  if (!bt || !ms_host || !launches_host) return SSA_INVALID_ARGUMENT;
  for (int k = 0; k < KIND_COUNT; ++k) {
    ms_host[k] = 0.0;
    launches_host[k] = 0;
  }
  if (!hip_ok(hipStreamSynchronize(bt->plan->stream))) return SSA_DEVICE_ERROR;
  for (size_t i = 0; i < bt->kinds.size(); ++i) {
    float ms = 0.f;
    if (!hip_ok(hipEventElapsedTime(&ms, bt->events[2 * i], bt->events[2 * i + 1])))
      return SSA_DEVICE_ERROR;
    ms_host[bt->kinds[i]] += ms;
    launches_host[bt->kinds[i]] += 1;
  }
  bt->kinds.clear();
  bt->ev_used = 0;
  bt->ev_error = false;
  return SSA_OK;
}

ssa_status ssa_batch_stats(ssa_batch *bt, ssa_stats *stats_host) {
  if (!bt || !stats_host) return SSA_INVALID_ARGUMENT;
  std::vector<dev_stats> h(bt->count);
  hipStream_t s = bt->plan->stream;
  if (!hip_ok(hipMemcpyAsync(h.data(), bt->stats, sizeof(dev_stats) * bt->count,
                             hipMemcpyDeviceToHost, s)) ||
      !hip_ok(hipStreamSynchronize(s)))
    return SSA_DEVICE_ERROR;
  for (size_t k = 0; k < bt->count; ++k)
    stats_host[bt->order[k]] = to_public(h[k], static_cast<int>(bt->h_tasks[k].log_n));
  return SSA_OK;
}

ssa_status ssa_mul_batch(ssa_plan *plan, size_t count, const uint8_t *const *a, const size_t *na,
                         const uint8_t *const *b, const size_t *nb, uint8_t *const *out,
                         int *status_dev) {
  ssa_batch *bt = nullptr;
  ssa_status r = ssa_batch_create(plan, count, a, na, b, nb, out, &bt);
  if (r != SSA_OK) return r;
  r = ssa_batch_run(bt, status_dev);
  if (r == SSA_OK && !hip_ok(hipStreamSynchronize(plan->stream))) r = SSA_DEVICE_ERROR;
  ssa_batch_destroy(bt);
  return r;
}

// ---------------------------------------------------------------------------
// Launch shapes and the autotuner

static launch_cfg from_public(const ssa_launch_config &c, int log_n, int pack, int arith) {
  launch_cfg r;
  r.log_n1 = c.log_n1;
  r.log_n2 = log_n - c.log_n1;
  r.cols = c.cols;
  r.rows = c.rows;
  r.pack = pack;
  r.persist = c.persistent;
  r.icols = c.inv_cols ? c.inv_cols : c.cols;
  r.arith = arith;
  return r;
}

ssa_status ssa_plan_get_config(const ssa_plan *plan, int log_n, ssa_launch_config *cfg) {
  if (!plan || !cfg || log_n <= SMALL_MAX_LOG || log_n > MAX_LOG_N) return SSA_INVALID_ARGUMENT;
  const launch_cfg &c = plan->cfg[log_n];
  *cfg = ssa_launch_config{c.log_n1, c.cols, c.rows, c.persist, c.icols};
  return SSA_OK;
}

ssa_status ssa_plan_set_config(ssa_plan *plan, int log_n, const ssa_launch_config *cfg) {
  if (!plan || !cfg || log_n <= SMALL_MAX_LOG || log_n > MAX_LOG_N) return SSA_INVALID_ARGUMENT;
  const launch_cfg c = from_public(*cfg, log_n, plan->opts.separate_transforms ? 0 : 1,
                                   plan->opts.arithmetic);
  if (!cfg_valid(c, log_n)) return SSA_INVALID_ARGUMENT;
  plan->cfg[log_n] = c;
  return SSA_OK;
}

ssa_status ssa_plan_autotune(ssa_plan *plan, int log_n, int count, ssa_launch_config *best,
                             double *best_ms_host, int *tried_host) {
  if (!plan || !best || !best_ms_host || log_n <= SMALL_MAX_LOG || log_n > plan->log_nmax ||
      count < 1 || count > 4096)
    return SSA_INVALID_ARGUMENT;
  // the digit size a multi-pass product of this plan runs in (the FP32 attempt
  // is single-workgroup, so with fp64_digit_bits every such product goes to
  // the FP64 path with those digits)
  const int bits = plan->opts.fp64_digit_bits ? plan->opts.fp64_digit_bits : plan->opts.digit_bits;
  const int pack = plan->opts.separate_transforms ? 0 : 1;
  const int arith = plan->opts.arithmetic;
  // equal operands as long as the plan allows, at most 2^(log_n - 1) digits each;
  // their transform length must be exactly 2^log_n
  const size_t nbytes = std::min(std::min(plan->max_na, plan->max_nb),
                                 (size_t(1) << (log_n - 1)) / (bits == 4 ? 2 : 1));
  if (log_n_for(2 * digits(nbytes, bits) - 1) != log_n) return SSA_INVALID_ARGUMENT;
  hipStream_t s = plan->stream;
  uint8_t *dops = nullptr, *dout = nullptr;
  const size_t ops_bytes = 2 * nbytes * count, out_bytes = 2 * nbytes * count;
  if (!hip_ok(hipMalloc(&dops, ops_bytes)) || !hip_ok(hipMalloc(&dout, out_bytes))) {
    (void)hipFree(dops);
    (void)hipGetLastError();
    return SSA_OUT_OF_MEMORY;
  }
  {  // pseudo-random operand bytes (xorshift), any content serves for timing
    std::vector<uint8_t> h(ops_bytes);
    uint64_t x = 0x9e3779b97f4a7c15ull;
    for (auto &b : h) {
      x ^= x << 13;
      x ^= x >> 7;
      x ^= x << 17;
      b = static_cast<uint8_t>(x >> 24);
    }
    if (!hip_ok(hipMemcpy(dops, h.data(), ops_bytes, hipMemcpyHostToDevice))) {
      (void)hipFree(dops);
      (void)hipFree(dout);
      return SSA_DEVICE_ERROR;
    }
  }
  std::vector<const uint8_t *> pa(count), pb(count);
  std::vector<uint8_t *> po(count);
  std::vector<size_t> na(count, nbytes), nb(count, nbytes);
  for (int i = 0; i < count; ++i) {
    pa[i] = dops + 2 * nbytes * i;
    pb[i] = dops + 2 * nbytes * i + nbytes;
    po[i] = dout + 2 * nbytes * i;
  }
  ssa_batch *bt = nullptr;
  ssa_status r = ssa_batch_create(plan, count, pa.data(), na.data(), pb.data(), nb.data(),
                                  po.data(), &bt);
  if (r == SSA_OK && (bt->h_tasks[0].log_n != static_cast<uint32_t>(log_n) || bt->bits[0] != bits)) {
    ssa_batch_destroy(bt);  // the products would not run at the length being tuned
    r = SSA_INVALID_ARGUMENT;
  }
  if (r != SSA_OK) {
    (void)hipFree(dops);
    (void)hipFree(dout);
    return r;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const launch_cfg keep = plan->cfg[log_n];
  launch_cfg bestc = keep;
  double bestms = 1e30;
  int tried = 0;
  bool ok = true;
  const auto time_shape = [&](const launch_cfg &c) {
    plan->cfg[log_n] = c;
    ok = hip_ok(enqueue_batch(bt, s, nullptr));  // warm-up
    if (!ok) return;
    const int reps = 8;  // shapes often differ by a few percent: average out the noise
    ok = hip_ok(hipEventRecord(e0, s));
    for (int k = 0; k < reps && ok; ++k) ok = hip_ok(enqueue_batch(bt, s, nullptr));
    ok = ok && hip_ok(hipEventRecord(e1, s)) && hip_ok(hipEventSynchronize(e1));
    float ms = 0.f;
    ok = ok && hip_ok(hipEventElapsedTime(&ms, e0, e1));
    ++tried;
    if (ok && ms / reps < bestms) {
      bestms = ms / reps;
      bestc = c;
    }
  };
  // every shape with one column count for both column passes; then, the rest of
  // the best shape kept, the inverse column pass's own count, and after it the
  // forward column pass's count (the two column passes are separate kernels, so
  // each search only moves its own pass's time)
  for (int l1 = 6; l1 <= 11 && ok; ++l1)
    for (int cols = 1; cols <= 32 && ok; cols *= 2)
      for (int rows = 1; rows <= 64 && ok; rows *= 2)
        for (int persist = 0; persist <= 1 && ok; ++persist) {
          const launch_cfg c{l1, log_n - l1, cols, rows, pack, persist, cols, arith};
          if (cfg_valid(c, log_n)) time_shape(c);
        }
  for (int pass = 0; pass < 2 && ok; ++pass) {
    const launch_cfg base = bestc;
    for (int k = 1; k <= 32 && ok; k *= 2) {
      launch_cfg c = base;
      (pass == 0 ? c.icols : c.cols) = k;
      if (k != (pass == 0 ? base.icols : base.cols) && cfg_valid(c, log_n)) time_shape(c);
    }
  }
  plan->cfg[log_n] = ok ? bestc : keep;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ssa_batch_destroy(bt);
  (void)hipFree(dops);
  (void)hipFree(dout);
  if (!ok) {
    (void)hipGetLastError();
    return SSA_DEVICE_ERROR;
  }
  *best = ssa_launch_config{bestc.log_n1, bestc.cols, bestc.rows, bestc.persist, bestc.icols};
  *best_ms_host = bestms;
  if (tried_host) *tried_host = tried;
  return SSA_OK;
}

}  // extern "C"
