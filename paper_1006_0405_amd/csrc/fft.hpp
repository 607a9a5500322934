// Building blocks of the interval DFT: global and LDS element access, the
// length-4 DFT (inner twiddles +-1, +-i are exact permutations in rectangular
// interval arithmetic, so they cause no wrapping) and the twiddle table.
#pragma once
#include "disc64.hpp"

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
typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
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
template <class E> __device__ __forceinline__ void radix4(E v[4]) {
  const E a = e_add(v[0], v[2]), b = e_sub(v[0], v[2]);
  const E c = e_add(v[1], v[3]), d = e_sub(v[1], v[3]);
  const E id = e_mul_i(d);
  v[0] = e_add(a, c);
  v[2] = e_sub(a, c);
  v[1] = e_add(b, id);
  v[3] = e_sub(b, id);
}

// Twiddle tables by level: tab[2^l + u] = omega_{2^l}^u (l <= log_ntab,
// u < 2^l) as point values (c, s) with a common absolute error bound e on each
// component.  The roots of one order are contiguous, so the twiddles of a
// length-2^l transform stay within a few cache lines.
struct twtab {
  const double2 *tab;
  int log_ntab;
  double e;
};
__device__ __forceinline__ double2 root(const twtab &T, int l, uint32_t u) {
  return T.tab[(1u << l) + u];
}
// The same levels copied into LDS (entries below 2^(l+1) for the levels a
// kernel uses), read through a local-address-space pointer so the reads are
// LDS instructions that never wait on global memory operations.
typedef __attribute__((address_space(3))) const double *lds_dp;
struct twtab_lds {
  lds_dp tab;  // 2 doubles (cos, sin) per entry
  int log_ntab;
  double e;
};
__device__ __forceinline__ double2 root(const twtab_lds &T, int l, uint32_t u) {
  const uint32_t i = 2u * ((1u << l) + u);
  return make_double2(T.tab[i], T.tab[i + 1]);
}

}  // namespace ssa
