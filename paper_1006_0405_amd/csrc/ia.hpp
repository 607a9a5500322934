// Interval arithmetic with outward rounding for gfx950 (CDNA4), device side.
//
// Containment sets (paper section 2.5): real intervals [lo, hi] and rectangular
// complex intervals [re] + i[im].  Every bound is produced by one IEEE
// operation rounded in the direction that keeps the true value inside.
//
// How the rounding direction is obtained on gfx950
// -------------------------------------------------
// VALU FP64 instructions have no per-instruction rounding field; they round
// according to the wave's MODE register.  A kernel calls enter_round_up() once:
// it sets the FP64 rounding field of MODE to "toward +infinity" for the rest of
// the wave.  Every interval bound is then an UPPER bound: a lower bound lo is
// stored negated, nlo = -lo, because RD(x) = -RU(-x).  With that layout
//   [a] + [b]:  nlo = RU(a.nlo + b.nlo),  hi = RU(a.hi + b.hi)
//   [a] - [b]:  nlo = RU(a.nlo + b.hi),   hi = RU(a.hi + b.nlo)
// and a product bound is the max of end-point products rounded up, so one
// rounding mode serves every operation and the mode is never switched back.
//
// The FP64 operations are written as inline assembly.  The compiler assumes
// round-to-nearest and would otherwise (a) fold -((-x)*y) into x*y, which is
// wrong under directed rounding, and (b) insert its own MODE resets before
// FP64 instructions it emits.  Assembly operands are opaque to both.  The
// assembly is not volatile, so it still schedules freely; its only inputs are
// values loaded after enter_round_up(), whose result (always 0) is folded into
// the kernel's base pointers so no FP64 operation can be hoisted above it.
//
// FP32 operations (the single-precision midpoint-radius path) are unaffected:
// enter_round_up() changes only the FP64/FP16 rounding field; FP32 stays at
// round-to-nearest-even.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ssa {

// Set FP64 rounding toward +infinity for this wave.  MODE[3:2] is the FP64/FP16
// rounding field (0 nearest-even, 1 +inf, 2 -inf, 3 zero).  The s_nop covers the
// wait states between a MODE write and dependent VALU instructions.
__device__ __forceinline__ uint32_t enter_round_up() {
  uint32_t z;
  asm volatile(
      "s_setreg_imm32_b32 hwreg(HW_REG_MODE, 2, 2), 1\n\t"
      "s_nop 3\n\t"
      "s_mov_b32 %0, 0"
      : "=s"(z)
      :
      : "memory");
  return z;
}

template <class T> __device__ __forceinline__ T *after_mode(T *p, uint32_t z) {
  return reinterpret_cast<T *>(reinterpret_cast<char *>(p) + z);
}
template <class T> __device__ __forceinline__ const T *after_mode(const T *p, uint32_t z) {
  return reinterpret_cast<const T *>(reinterpret_cast<const char *>(p) + z);
}

// ---- FP64 operations, rounded toward +inf (valid after enter_round_up) ----
__device__ __forceinline__ double ru_add(double a, double b) {
  double r;
  asm("v_add_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ double ru_mul(double a, double b) {
  double r;
  asm("v_mul_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
// RU(-a * b): the negation is a source modifier, exact.
__device__ __forceinline__ double ru_nmul(double a, double b) {
  double r;
  asm("v_mul_f64 %0, -%1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
// RU(a * b + c), one rounding.
__device__ __forceinline__ double ru_fma(double a, double b, double c) {
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}
// Operations that do not round (exact in any mode).
__device__ __forceinline__ double dmax(double a, double b) {
  double r;
  asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ double dfloor(double a) {
  double r;
  asm("v_floor_f64 %0, %1" : "=v"(r) : "v"(a));
  return r;
}
__device__ __forceinline__ double dabs(double a) {
  return __longlong_as_double(__double_as_longlong(a) & 0x7fffffffffffffffLL);
}
__device__ __forceinline__ bool sign_clear(double a) {
  return __double_as_longlong(a) >= 0;  // +0 and positive values
}

// ---- Rectangular complex interval, lower bounds negated --------------------
// re in [-rn, rh], im in [-in, ih].  32 bytes, the unit of every FFT array.
struct alignas(16) ci {
  double rn, rh, in, ih;
};

__device__ __forceinline__ ci ci_thin_real(double v) { return ci{-v, v, 0.0, 0.0}; }

__device__ __forceinline__ ci ci_add(const ci &a, const ci &b) {
  return ci{ru_add(a.rn, b.rn), ru_add(a.rh, b.rh), ru_add(a.in, b.in), ru_add(a.ih, b.ih)};
}
__device__ __forceinline__ ci ci_sub(const ci &a, const ci &b) {
  return ci{ru_add(a.rn, b.rh), ru_add(a.rh, b.rn), ru_add(a.in, b.ih), ru_add(a.ih, b.in)};
}
// i * z: re = -im, im = re (exact permutation).
__device__ __forceinline__ ci ci_mul_i(const ci &a) { return ci{a.ih, a.in, a.rn, a.rh}; }
// -i * z: re = im, im = -re.
__device__ __forceinline__ ci ci_mul_negi(const ci &a) { return ci{a.in, a.ih, a.rh, a.rn}; }
// complex conjugate (exact).
__device__ __forceinline__ ci ci_conj(const ci &a) { return ci{a.rn, a.rh, a.ih, a.in}; }

// Multiplication by a root of unity w, known as a point (c, s) with
// |Re w - c| <= e and |Im w - s| <= e.  For x in [x], y in [y]:
//   Re(w z) = c x - s y + (dc x - ds y),  |dc x - ds y| <= e (|x|max + |y|max)
//   Im(w z) = s x + c y + (ds x + dc y),  same bound,
// and for a point factor c the interval c[x] is [c x.lo, c x.hi] (c >= 0) or
// [c x.hi, c x.lo] (c < 0).  Each bound is then one fused chain rounded up.
// This encloses the paper's rectangular product [w][z] (section 2.5) with the
// twiddle's rounding error folded into a common radius term.
__device__ __forceinline__ ci ci_twiddle(const ci &z, double c, double s, double e) {
  const double ac = dabs(c), as = dabs(s);
  const bool cp = sign_clear(c), sp = sign_clear(s);
  const double mx = dmax(z.rn, z.rh), my = dmax(z.in, z.ih);
  const double E = ru_mul(e, ru_add(mx, my));
  const double xh_c = cp ? z.rh : z.rn, xn_c = cp ? z.rn : z.rh;
  const double yh_c = cp ? z.ih : z.in, yn_c = cp ? z.in : z.ih;
  const double xh_s = sp ? z.rh : z.rn, xn_s = sp ? z.rn : z.rh;
  const double yh_s = sp ? z.ih : z.in, yn_s = sp ? z.in : z.ih;
  ci r;
  r.rh = ru_fma(ac, xh_c, ru_fma(as, yn_s, E));  // c x - s y, upper
  r.rn = ru_fma(ac, xn_c, ru_fma(as, yh_s, E));  // -(c x - s y), upper
  r.ih = ru_fma(as, xh_s, ru_fma(ac, yh_c, E));  // s x + c y, upper
  r.in = ru_fma(as, xn_s, ru_fma(ac, yn_c, E));  // -(s x + c y), upper
  return r;
}

// Real interval product (paper section 2.5, four end-point products): with
// x = [-xn, xh], y = [-yn, yh] the end-point products are xn*yn, -xn*yh,
// -xh*yn, xh*yh; hi = max of them rounded up, nlo = max of their negatives
// rounded up.
struct ri {
  double n, h;
};
__device__ __forceinline__ ri ri_mul(double xn, double xh, double yn, double yh) {
  const double h = dmax(dmax(ru_mul(xn, yn), ru_nmul(xn, yh)), dmax(ru_nmul(xh, yn), ru_mul(xh, yh)));
  const double n = dmax(dmax(ru_nmul(xn, yn), ru_mul(xn, yh)), dmax(ru_mul(xh, yn), ru_nmul(xh, yh)));
  return ri{n, h};
}
// Complex interval product (paper section 2.5):
// ([z1][w1] - [z2][w2]) + i([z1][w2] + [z2][w1]).
__device__ __forceinline__ ci ci_mul(const ci &z, const ci &w) {
  const ri a = ri_mul(z.rn, z.rh, w.rn, w.rh);  // z1 w1
  const ri b = ri_mul(z.in, z.ih, w.in, w.ih);  // z2 w2
  const ri c = ri_mul(z.rn, z.rh, w.in, w.ih);  // z1 w2
  const ri d = ri_mul(z.in, z.ih, w.rn, w.rh);  // z2 w1
  return ci{ru_add(a.n, b.h), ru_add(a.h, b.n), ru_add(c.n, d.n), ru_add(c.h, d.h)};
}

// Multiplication of every bound by 2^-k (exact unless it underflows; rounding
// up keeps both stored bounds valid either way).
__device__ __forceinline__ ci ci_scale(const ci &a, double p2) {
  return ci{ru_mul(a.rn, p2), ru_mul(a.rh, p2), ru_mul(a.in, p2), ru_mul(a.ih, p2)};
}

}  // namespace ssa
