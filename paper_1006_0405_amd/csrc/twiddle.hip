// Certified twiddle table, generated on the GPU.
//
// The roots omega_{2^s} = e^{2 pi i / 2^s} come from the half-angle recurrence
// of paper section 2.2:  omega_1 = 1, omega_2 = -1, omega_4 = i and
// omega_{2n} = (1 + omega_n) / |1 + omega_n|,  evaluated in interval
// arithmetic with the square root and division of section 2.5.  The powers
// omega_N^t are products over the set bits of t:  omega_N^{2^b} = omega_{2^{K-b}}.
//
// All of it runs in exact integer arithmetic on fixed-point numbers with 62
// fractional bits (value = X / 2^62), each bound rounded outward by floor/ceil
// of an exact 128-bit quantity, so the enclosures are rigorous without any
// floating-point rounding-mode dependence, and about 2^-55 wide instead of the
// hundreds of ulps that the same products accumulate in rectangular double
// intervals.  Each entry is then stored as the double nearest its midpoint,
// and the largest distance from any stored component to the end of its
// enclosure (computed exactly, converted to double rounding up) becomes the
// table's single error bound e:  |Re omega_N^t - c_t| <= e, |Im omega_N^t - s_t| <= e.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "twiddle.hpp"

namespace ssa {

typedef __int128 i128;
typedef unsigned __int128 u128;

static constexpr int FB = 62;              // fractional bits
static constexpr int64_t ONE = int64_t(1) << FB;

struct fi {  // fixed-point interval [lo, hi] (scaled by 2^62)
  int64_t lo, hi;
};
struct fc {  // fixed-point rectangular complex interval
  fi re, im;
};

__device__ __forceinline__ int64_t shr_floor(i128 x) { return static_cast<int64_t>(x >> FB); }
__device__ __forceinline__ int64_t shr_ceil(i128 x) { return -static_cast<int64_t>((-x) >> FB); }

__device__ __forceinline__ i128 imin(i128 a, i128 b) { return a < b ? a : b; }
__device__ __forceinline__ i128 imax(i128 a, i128 b) { return a > b ? a : b; }

// Exact end-point products of two intervals (scaled by 2^124).
struct p124 {
  i128 lo, hi;
};
__device__ __forceinline__ p124 fprod(fi a, fi b) {
  const i128 p1 = (i128)a.lo * b.lo, p2 = (i128)a.lo * b.hi;
  const i128 p3 = (i128)a.hi * b.lo, p4 = (i128)a.hi * b.hi;
  return p124{imin(imin(p1, p2), imin(p3, p4)), imax(imax(p1, p2), imax(p3, p4))};
}

// Rectangular complex interval product, one outward rounding per bound.
__device__ __forceinline__ fc fcmul(const fc &z, const fc &w) {
  const p124 a = fprod(z.re, w.re), b = fprod(z.im, w.im);
  const p124 c = fprod(z.re, w.im), d = fprod(z.im, w.re);
  fc r;
  r.re.lo = shr_floor(a.lo - b.hi);
  r.re.hi = shr_ceil(a.hi - b.lo);
  r.im.lo = shr_floor(c.lo + d.lo);
  r.im.hi = shr_ceil(c.hi + d.hi);
  return r;
}

// floor(sqrt(v)) for v < 2^127.
__device__ uint64_t isqrt_floor(u128 v) {
  if (v == 0) return 0;
  const double vd = static_cast<double>(static_cast<uint64_t>(v >> 64)) * 18446744073709551616.0 +
                    static_cast<double>(static_cast<uint64_t>(v));
  uint64_t r = static_cast<uint64_t>(sqrt(vd));
  for (int it = 0; it < 3; ++it) {  // integer Newton steps from the estimate
    if (r == 0) r = 1;
    const u128 q = v / r;
    r = static_cast<uint64_t>((static_cast<u128>(r) + q) >> 1);
  }
  while (static_cast<u128>(r) * r > v) --r;
  while (static_cast<u128>(r + 1) * (r + 1) <= v) ++r;
  return r;
}

__global__ void k_roots(int K, fc *roots) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  fc R;
  R = fc{{ONE, ONE}, {0, 0}};
  roots[0] = R;
  if (K >= 1) roots[1] = fc{{-ONE, -ONE}, {0, 0}};
  if (K >= 2) roots[2] = fc{{0, 0}, {ONE, ONE}};
  R = fc{{0, 0}, {ONE, ONE}};
  for (int s = 2; s < K; ++s) {
    // For s >= 2 both components of omega_{2^s} are >= 0, so 1 + Re >= 1 and
    // the squares and quotients below are monotone in each bound.
    const u128 nre_lo = (u128)(ONE + (i128)R.re.lo), nre_hi = (u128)(ONE + (i128)R.re.hi);
    const u128 nim_lo = (u128)R.im.lo, nim_hi = (u128)R.im.hi;
    const u128 sq_lo = nre_lo * nre_lo + nim_lo * nim_lo;  // < 2^127
    const u128 sq_hi = nre_hi * nre_hi + nim_hi * nim_hi;
    // |1 + omega| enclosed by [floor sqrt(sq_lo), ceil sqrt(sq_hi)] (scale 2^62)
    const uint64_t m_lo = isqrt_floor(sq_lo);
    uint64_t m_hi = isqrt_floor(sq_hi);
    if ((u128)m_hi * m_hi < sq_hi) ++m_hi;
    // component / magnitude: [lo / m_hi, hi / m_lo], rounded outward
    fc Rn;
    const u128 nl = nre_lo << FB, nh = nre_hi << FB;
    const u128 il = nim_lo << FB, ih = nim_hi << FB;
    Rn.re.lo = static_cast<int64_t>(nl / m_hi);
    Rn.re.hi = static_cast<int64_t>(nh / m_lo + ((nh % m_lo) != 0));
    Rn.im.lo = static_cast<int64_t>(il / m_hi);
    Rn.im.hi = static_cast<int64_t>(ih / m_lo + ((ih % m_lo) != 0));
    R = Rn;
    roots[s + 1] = R;
  }
}

// x / 2^scale as a double rounded up (x >= 0).
__device__ double u128_to_double_up(u128 x, int scale) {
  if (x == 0) return 0.0;
  int p = 127;
  while (!((x >> p) & 1)) --p;
  uint64_t mant;
  int shift = 0;
  if (p <= 52) {
    mant = static_cast<uint64_t>(x);
  } else {
    shift = p - 52;
    mant = static_cast<uint64_t>(x >> shift);
    const u128 rest = x - (static_cast<u128>(mant) << shift);
    if (rest != 0) ++mant;  // round up; 2^53 is still exact
  }
  return ldexp(static_cast<double>(mant), shift - scale);
}

// Exact value of a double as a signed integer scaled by 2^120.  Every double
// produced below has magnitude >= 2^-62 or is 0, so the product is an integer.
__device__ i128 double_to_fx120(double d) {
  if (d == 0.0) return 0;
  const int64_t bits = __double_as_longlong(d);
  const int exp = static_cast<int>((bits >> 52) & 0x7ff) - 1075;  // d = m * 2^exp
  const int64_t m = (bits & ((int64_t(1) << 52) - 1)) | (int64_t(1) << 52);
  const int sh = exp + 120;
  i128 v = sh >= 0 ? ((i128)m << sh) : ((i128)m >> (-sh));
  return bits < 0 ? -v : v;
}

// Stores the double nearest the midpoint of [lo, hi]; returns an upper bound
// of the distance from it to either end (the true value lies in between).
__device__ double midpoint_and_error(fi x, double *out) {
  const int64_t mid = (x.lo >> 1) + (x.hi >> 1) + (x.lo & x.hi & 1);
  const double c = ldexp(static_cast<double>(mid), -FB);
  *out = c;
  const i128 c120 = double_to_fx120(c);
  const i128 lo120 = (i128)x.lo << 58, hi120 = (i128)x.hi << 58;
  const i128 d1 = hi120 - c120, d2 = c120 - lo120;
  const i128 d = d1 > d2 ? d1 : d2;
  return u128_to_double_up(static_cast<u128>(d < 0 ? 0 : d), 120);
}

__global__ void k_table(int K, const fc *roots, double2 *tab, unsigned long long *ebits) {
  const uint32_t N = 1u << K;
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  double emax = 0.0;
  if (t < N) {
    fc T{{ONE, ONE}, {0, 0}};
    for (int b = 0; b < K; ++b)
      if ((t >> b) & 1u) T = fcmul(T, roots[K - b]);
    double c, s;
    const double ec = midpoint_and_error(T.re, &c);
    const double es = midpoint_and_error(T.im, &s);
    tab[t] = make_double2(c, s);
    emax = ec > es ? ec : es;
  }
  // block maximum, then one atomic per block (non-negative doubles order like
  // their bit patterns)
  __shared__ unsigned long long sm;
  if (threadIdx.x == 0) sm = 0;
  __syncthreads();
  atomicMax(&sm, static_cast<unsigned long long>(__double_as_longlong(emax)));
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(ebits, sm);
}

hipError_t make_twiddles(int K, double2 *tab, unsigned long long *ebits, void *roots_scratch,
                         hipStream_t stream) {
  fc *roots = static_cast<fc *>(roots_scratch);
  hipLaunchKernelGGL(k_roots, dim3(1), dim3(64), 0, stream, K, roots);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  const uint32_t N = 1u << K;
  const uint32_t bs = 256;
  hipLaunchKernelGGL(k_table, dim3((N + bs - 1) / bs), dim3(bs), 0, stream, K, roots, tab, ebits);
  return hipGetLastError();
}

size_t twiddle_roots_bytes() { return sizeof(fc) * 64; }

__global__ void k_levels(int K, double2 *lv) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (1u << K)) return;
  if (i == 0) {
    lv[0] = make_double2(1.0, 0.0);  // unused slot
    return;
  }
  const int l = 31 - __builtin_clz(i);
  const uint32_t u = i - (1u << l);
  lv[i] = lv[(1u << K) + (u << (K - l))];
}

hipError_t make_level_tables(int K, double2 *lv, hipStream_t stream) {
  const uint32_t n = 1u << K;
  const uint32_t bs = 256;
  hipLaunchKernelGGL(k_levels, dim3((n + bs - 1) / bs), dim3(bs), 0, stream, K, lv);
  return hipGetLastError();
}

}  // namespace ssa
