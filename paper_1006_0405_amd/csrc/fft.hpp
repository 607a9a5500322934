// Interval DFT of length M = 2^m computed cooperatively by the M/4 threads of a
// thread group, data in registers, exchanges through LDS.
//
// The transform is the DFT of the paper (section 2.2) with omega = e^{+2 pi i/M}.
// Instead of the recursive radix-2 Cooley-Tukey box it uses the Stockham
// (self-sorting) formulation of the same factorisation with radix 4 (and one
// radix-2 stage when m is odd): input and output are in natural order, every
// stage reads the group's elements with unit stride (coalesced from global
// memory on the first stage, conflict-light in LDS afterwards), and the radix-4
// kernel's inner twiddles are +-1 and +-i, which are exact in rectangular
// interval arithmetic (no wrapping), so only one twiddle multiplication per
// element and per two levels is interval-inexact.
//
// Stage s with radix R and Ns = product of the earlier radices: thread j takes
// v_r = x[j + r M/R], multiplies v_r by omega_{R Ns}^{r k} (k = j mod Ns), applies
// the length-R DFT and writes result q to y[(j - k) R + k + q Ns].  After the
// last stage (R Ns = M) result q of thread j is X[j + q M/4], already in the
// thread's own registers.
#pragma once
#include "ia.hpp"

namespace ssa {

// One complex interval element in LDS: two 16-byte halves.
__device__ __forceinline__ void lds_put(ci *lds, int idx, const ci &v) {
  double2 *p = reinterpret_cast<double2 *>(lds + idx);
  p[0] = make_double2(v.rn, v.rh);
  p[1] = make_double2(v.in, v.ih);
}
__device__ __forceinline__ ci lds_get(const ci *lds, int idx) {
  const double2 *p = reinterpret_cast<const double2 *>(lds + idx);
  const double2 a = p[0], b = p[1];
  return ci{a.x, a.y, b.x, b.y};
}
// Global-memory accesses through address-space-1 pointers, so that the
// compiler emits global (not flat) loads and stores for pointers that came out
// of a descriptor in memory.
typedef double d2v __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) const d2v *gcd2;
typedef __attribute__((address_space(1))) d2v *gd2;
__device__ __forceinline__ ci gld(const ci *g, size_t idx) {
  const gcd2 p = reinterpret_cast<gcd2>(reinterpret_cast<uintptr_t>(g + idx));
  const d2v a = p[0], b = p[1];
  return ci{a.x, a.y, b.x, b.y};
}
__device__ __forceinline__ void gst(ci *g, size_t idx, const ci &v) {
  const gd2 p = reinterpret_cast<gd2>(reinterpret_cast<uintptr_t>(g + idx));
  p[0] = d2v{v.rn, v.rh};
  p[1] = d2v{v.in, v.ih};
}

template <class T> __device__ __forceinline__ T gload(const T *p) {
  return *reinterpret_cast<__attribute__((address_space(1))) const T *>(reinterpret_cast<uintptr_t>(p));
}
template <class T> __device__ __forceinline__ void gstore(T *p, T v) {
  *reinterpret_cast<__attribute__((address_space(1))) T *>(reinterpret_cast<uintptr_t>(p)) = v;
}

// Length-4 DFT with omega_4 = +i:  y0 = a + c, y2 = a - c, y1 = b + i d,
// y3 = b - i d, where a = v0 + v2, b = v0 - v2, c = v1 + v3, d = v1 - v3.
__device__ __forceinline__ void radix4(ci v[4]) {
  const ci a = ci_add(v[0], v[2]), b = ci_sub(v[0], v[2]);
  const ci c = ci_add(v[1], v[3]), d = ci_sub(v[1], v[3]);
  const ci id = ci_mul_i(d);
  v[0] = ci_add(a, c);
  v[2] = ci_sub(a, c);
  v[1] = ci_add(b, id);
  v[3] = ci_sub(b, id);
}

// Twiddle table: omega_{Ntab}^t for 0 <= t < Ntab as point values (c, s) with
// a common absolute error bound e on each component.
struct twtab {
  const double2 *tab;
  int log_ntab;
  double e;
};

__device__ __forceinline__ ci apply_tw(const ci &v, const twtab &T, uint32_t t) {
  const double2 w = T.tab[t];
  return ci_twiddle(v, w.x, w.y, T.e);
}

// Forward interval DFT of the group's M elements.  `lds` points at element 0
// of this group's exchange buffer; element i lives at lds[i * is].  All threads
// of the workgroup must call this with the same M (it contains barriers).
__device__ __forceinline__ void fft_group(ci v[4], int j, int logM, ci *lds, int is,
                                          const twtab &T) {
  const int M = 1 << logM;
  const int Q = M >> 2;
  int logNs = 0;
  if (logM & 1) {
    // Radix-2 stage with Ns = 1 (no twiddles).  This thread acts for the two
    // radix-2 positions j (pair v0, v2) and j + M/4 (pair v1, v3).
    const ci a0 = ci_add(v[0], v[2]), a1 = ci_sub(v[0], v[2]);
    const ci b0 = ci_add(v[1], v[3]), b1 = ci_sub(v[1], v[3]);
    __syncthreads();
    lds_put(lds, (2 * j) * is, a0);
    lds_put(lds, (2 * j + 1) * is, a1);
    lds_put(lds, (2 * j + 2 * Q) * is, b0);
    lds_put(lds, (2 * j + 2 * Q + 1) * is, b1);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = lds_get(lds, (j + r * Q) * is);
    logNs = 1;
  }
  for (;;) {
    const int Ns = 1 << logNs;
    const int k = j & (Ns - 1);
    if (logNs > 0) {
      const int sh = T.log_ntab - (logNs + 2);
#pragma unroll
      for (int r = 1; r < 4; ++r) v[r] = apply_tw(v[r], T, static_cast<uint32_t>(r * k) << sh);
    }
    radix4(v);
    if (logNs + 2 == logM) break;  // last stage: X[j + q M/4] = v[q]
    const int base = ((j - k) << 2) + k;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) lds_put(lds, (base + q * Ns) * is, v[q]);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = lds_get(lds, (j + r * Q) * is);
    logNs += 2;
  }
}

}  // namespace ssa
