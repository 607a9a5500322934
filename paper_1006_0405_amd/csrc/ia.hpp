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
//   Im(w z) = s x + c y + (ds x + dc y),  same bound.
// A point factor is split by sign, c = c+ - c- with c+ = max(c, 0) and
// c- = max(-c, 0) (one of them is 0), so that without any branch or select
//   hi(c [x])  = c+ x.hi + c- (-x.lo)   and   -lo(c [x]) = c+ (-x.lo) + c- x.hi,
// and every bound is one fused chain rounded up.  This encloses the paper's
// rectangular product [w][z] (section 2.5) with the twiddle's rounding error
// folded into a common radius term.
__device__ __forceinline__ ci ci_twiddle(const ci &z, double c, double s, double e) {
  const double cp = dmax(c, 0.0), cn = dmax(-c, 0.0);
  const double sp = dmax(s, 0.0), sn = dmax(-s, 0.0);
  const double mx = dmax(z.rn, z.rh), my = dmax(z.in, z.ih);
  const double E = ru_mul(e, ru_add(mx, my));
  ci r;
  // Re = c x - s y:  hi = hi(c x) + (-lo(s y)),  -lo = -lo(c x) + hi(s y)
  r.rh = ru_fma(cp, z.rh, ru_fma(cn, z.rn, ru_fma(sp, z.in, ru_fma(sn, z.ih, E))));
  r.rn = ru_fma(cp, z.rn, ru_fma(cn, z.rh, ru_fma(sp, z.ih, ru_fma(sn, z.in, E))));
  // Im = s x + c y:  hi = hi(s x) + hi(c y),  -lo = -lo(s x) + (-lo(c y))
  r.ih = ru_fma(sp, z.rh, ru_fma(sn, z.rn, ru_fma(cp, z.ih, ru_fma(cn, z.in, E))));
  r.in = ru_fma(sp, z.rn, ru_fma(sn, z.rh, ru_fma(cp, z.in, ru_fma(cn, z.ih, E))));
  return r;
}

// The product of two stored roots w1 = (c1, s1), w2 = (c2, s2) (each within e
// of the true root componentwise) as a point (c, s) with its own bound:
// the exact product of the stored points lies in [-re_n, re_h] x [-im_n, im_h]
// (bounds rounded up), and the true roots' product differs from it by at most
// e (|c1| + |s1| + |c2| + |s2|) + 2 e^2 per component.
struct twpoint {
  double c, s, e;
};
__device__ __forceinline__ twpoint tw_product(double2 w1, double2 w2, double e) {
  const double re_h = ru_fma(w1.x, w2.x, ru_nmul(w1.y, w2.y));
  const double re_n = ru_fma(-w1.x, w2.x, ru_mul(w1.y, w2.y));
  const double im_h = ru_fma(w1.x, w2.y, ru_mul(w1.y, w2.x));
  const double im_n = ru_fma(-w1.x, w2.y, ru_nmul(w1.y, w2.x));
  const double l1 = ru_add(ru_add(dabs(w1.x), dabs(w1.y)), ru_add(dabs(w2.x), dabs(w2.y)));
  const double E2 = ru_fma(e, l1, ru_mul(ru_add(e, e), e));
  const double ec = ru_add(ru_add(re_h, re_n), E2), es = ru_add(ru_add(im_h, im_n), E2);
  return twpoint{re_h, im_h, dmax(ec, es)};
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
