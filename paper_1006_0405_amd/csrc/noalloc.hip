// ssa_mul_noalloc: the product of ssa_mul without any allocation, for callers
// that cannot allocate device memory (code under HIP graph capture, serving
// loops, harnesses that forbid hipMalloc).
//
// Everything ssa_mul keeps in a plan -- the certified twiddle table, the
// transform array, the coefficients, the statistics, the carry-scan status
// words and the product's descriptor -- lives in one file-scope device array
// (`scratch`) of a fixed size, enough for transforms of up to 2^NA_LOG_N
// points.  Each device holds its own copy at its own address, found once per
// device with hipGetSymbolAddress; host code uses only that address.  The
// first call on a device also builds the twiddle table there and reads back
// its error bound; later calls enqueue kernels only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "../../include/ssa.h"
#include "internal.hpp"
#include "twiddle.hpp"

using namespace ssa;

namespace {

constexpr int NA_LOG_N = 18;  // largest transform: L = na + nb - 1 <= 2^18 coefficients
constexpr size_t NA_N = size_t(1) << NA_LOG_N;
constexpr size_t round256(size_t x) { return (x + 255) & ~size_t(255); }
// na + nb <= L + 1 <= 2^18 + 1 product bytes
constexpr size_t NA_MAX_TILES = (NA_N + 1 + CARRY_TILE - 1) / CARRY_TILE;
constexpr size_t NA_ROOTS_BYTES = 4096;

// Layout of the array (byte offsets, 256-byte aligned).
constexpr size_t OFF_TAB = 0;  // level tables, 2^(NA_LOG_N + 1) double2
constexpr size_t OFF_Y = OFF_TAB + round256(sizeof(double2) * 2 * NA_N);  // transform array
constexpr size_t OFF_C = OFF_Y + round256(sizeof(ci) * NA_N);             // coefficients
constexpr size_t OFF_TILES = OFF_C + round256(sizeof(unsigned long long) * NA_N);
constexpr size_t OFF_ST = OFF_TILES + round256(sizeof(uint32_t) * TILE_WORD_STRIDE * NA_MAX_TILES);
constexpr size_t OFF_TASK = OFF_ST + round256(sizeof(dev_stats));
constexpr size_t OFF_EBITS = OFF_TASK + round256(sizeof(task));
constexpr size_t OFF_ROOTS = OFF_EBITS + 256;
constexpr size_t SCRATCH_BYTES = OFF_ROOTS + NA_ROOTS_BYTES;  // about 18.1 MiB

}  // namespace

// The scratch array (one copy per device).  In host code its name stands for
// a host-side shadow, not for device memory: host code passes only the
// address hipGetSymbolAddress returns for it on the current device.
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
struct device_scratch {
  unsigned char *ptr = nullptr;  // device address of `scratch` on that device
  double e = 0.0;                // error bound of the twiddle table built there
};
std::mutex g_mu;
device_scratch g_dev[MAX_DEVICES];

// The product's descriptor, passed by value (a kernel argument, so a captured
// launch keeps its own copy) and written into the array.
__global__ void k_put_task(task t, task *dst) { *dst = t; }

// Once per device, with that device current: find the array, build the
// twiddle table in it and read back its bound.
ssa_status init_device(int dev, hipStream_t s) {
  if (twiddle_roots_bytes() > NA_ROOTS_BYTES) return SSA_INTERNAL_ERROR;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess) return SSA_DEVICE_ERROR;
  if (cs != hipStreamCaptureStatusNone) return SSA_INVALID_ARGUMENT;  // must not be captured
  void *p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) {
    (void)hipGetLastError();
    return SSA_DEVICE_ERROR;
  }
  unsigned char *base = static_cast<unsigned char *>(p);
  double2 *tab = reinterpret_cast<double2 *>(base + OFF_TAB);
  unsigned long long *ebits = reinterpret_cast<unsigned long long *>(base + OFF_EBITS);
  unsigned long long eb = 0;
  const bool ok = set_kernel_attributes() == hipSuccess &&
                  hipMemsetAsync(ebits, 0, sizeof(eb), s) == hipSuccess &&
                  make_twiddles(NA_LOG_N, tab + NA_N, ebits, base + OFF_ROOTS, s) == hipSuccess &&
                  make_level_tables(NA_LOG_N, tab, s) == hipSuccess &&
                  hipMemcpyAsync(&eb, ebits, sizeof(eb), hipMemcpyDeviceToHost, s) == hipSuccess &&
                  hipStreamSynchronize(s) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    return SSA_DEVICE_ERROR;
  }
  std::memcpy(&g_dev[dev].e, &eb, sizeof(double));
  g_dev[dev].ptr = base;
  return SSA_OK;
}

int ceil_log2(uint64_t v) {
  int k = 0;
  while ((uint64_t(1) << k) < v) ++k;
  return k;
}

}  // namespace

extern "C" ssa_status ssa_mul_noalloc(const uint8_t *a, size_t na, const uint8_t *b, size_t nb,
                                      uint8_t *out, int *status_dev, void *stream) {
  if (!a || !b || !out || !status_dev || na == 0 || nb == 0 || na > NA_N || nb > NA_N ||
      na + nb - 1 > NA_N)
    return SSA_INVALID_ARGUMENT;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return SSA_DEVICE_ERROR;
  device_scratch d;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_dev[dev].ptr == nullptr) {
      const ssa_status r = init_device(dev, s);
      if (r != SSA_OK) return r;
    }
    d = g_dev[dev];
  }
  const uint64_t L = uint64_t(na) + nb - 1;
  const int log_n = std::max(ceil_log2(L), SMALL_MIN_LOG);
  task t;
  std::memset(&t, 0, sizeof(t));
  t.a = a;
  t.b = b;
  t.out = out;
  t.na = t.nda = static_cast<uint32_t>(na);
  t.nb = t.ndb = static_cast<uint32_t>(nb);
  t.L = static_cast<uint32_t>(L);
  t.log_n = static_cast<uint32_t>(log_n);
  t.ya = reinterpret_cast<ci *>(d.ptr + OFF_Y);
  t.yb = nullptr;  // packed transform: one array
  t.c = reinterpret_cast<unsigned long long *>(d.ptr + OFF_C);
  t.st = reinterpret_cast<dev_stats *>(d.ptr + OFF_ST);
  t.tiles = reinterpret_cast<uint32_t *>(d.ptr + OFF_TILES);
  t.ntiles = static_cast<uint32_t>((na + nb + CARRY_TILE - 1) / CARRY_TILE);
  t.fp32 = 0u;
  task *d_task = reinterpret_cast<task *>(d.ptr + OFF_TASK);
  const twtab_host tw{reinterpret_cast<const double2 *>(d.ptr + OFF_TAB), NA_LOG_N, d.e};
  hipLaunchKernelGGL(k_put_task, dim3(1), dim3(1), 0, s, t, d_task);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    if (log_n <= SMALL_MAX_LOG) {
      e = launch_small(d_task, 1, log_n, 8, CERT_ONE_INTEGER, 1, ARITH_RECT, 0, 0, 0, tw, nullptr,
                       s);
    } else {
      e = launch_multipass(d_task, 1, log_n, default_launch_cfg(log_n, 1, ARITH_RECT), 8,
                           CERT_ONE_INTEGER, tw, nullptr, s);
      if (e == hipSuccess) e = launch_carry(d_task, 1, t.ntiles, 8, s);
    }
  }
  if (e == hipSuccess) e = launch_status(d_task, 1, status_dev, s);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return SSA_DEVICE_ERROR;
  }
  return SSA_OK;
}
