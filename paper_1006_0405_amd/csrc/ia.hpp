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
// RU(a - b), RU(-a * b + c), RU(a * b - c), RU(a * |b| + c), RU(|a| + b):
// negations and absolute values are source modifiers, exact.
__device__ __forceinline__ double ru_sub(double a, double b) {
  double r;
  asm("v_add_f64 %0, %1, -%2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ double ru_nfma(double a, double b, double c) {
  double r;
  asm("v_fma_f64 %0, -%1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}
__device__ __forceinline__ double ru_fms(double a, double b, double c) {
  double r;
  asm("v_fma_f64 %0, %1, %2, -%3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}
__device__ __forceinline__ double ru_fma_ab(double a, double b, double c) {
  double r;
  asm("v_fma_f64 %0, %1, |%2|, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}
__device__ __forceinline__ double ru_mul_ab(double a, double b) {
  double r;
  asm("v_mul_f64 %0, %1, |%2|" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ double ru_add_aa(double a, double b) {
  double r;
  asm("v_add_f64 %0, |%1|, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
// Operations that do not round (exact in any mode).
__device__ __forceinline__ double dmax(double a, double b) {
  double r;
  asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
// Positive and negative parts max(a, 0) and max(-a, 0) (exact; the negation is
// a source modifier and 0 an inline constant).
__device__ __forceinline__ double dpos(double a) {
  double r;
  asm("v_max_f64 %0, %1, 0" : "=v"(r) : "v"(a));
  return r;
}
__device__ __forceinline__ double dneg(double a) {
  double r;
  asm("v_max_f64 %0, -%1, 0" : "=v"(r) : "v"(a));
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
// re in [-rn, rh], im in [-in, ih].  32 bytes in registers and in the
// standalone transform's arrays; the product's arrays between passes keep a
// midpoint and one radius instead (20 bytes).
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
  const double cp = dpos(c), cn = dneg(c);
  const double sp = dpos(s), sn = dneg(s);
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

// Known-sign forms of ci_twiddle, for roots whose stored point is known to lie
// in the closed first quadrant (c >= 0, s >= 0) or upper half plane (s >= 0):
// the terms with the zero half of the sign split are dropped.
__device__ __forceinline__ ci ci_twiddle_q1(const ci &z, double c, double s, double e) {
  const double mx = dmax(z.rn, z.rh), my = dmax(z.in, z.ih);
  const double E = ru_mul(e, ru_add(mx, my));
  ci r;
  r.rh = ru_fma(c, z.rh, ru_fma(s, z.in, E));
  r.rn = ru_fma(c, z.rn, ru_fma(s, z.ih, E));
  r.ih = ru_fma(s, z.rh, ru_fma(c, z.ih, E));
  r.in = ru_fma(s, z.rn, ru_fma(c, z.in, E));
  return r;
}
__device__ __forceinline__ ci ci_twiddle_uh(const ci &z, double c, double s, double e) {
  const double cp = dpos(c), cn = dneg(c);
  const double mx = dmax(z.rn, z.rh), my = dmax(z.in, z.ih);
  const double E = ru_mul(e, ru_add(mx, my));
  ci r;
  r.rh = ru_fma(cp, z.rh, ru_fma(cn, z.rn, ru_fma(s, z.in, E)));
  r.rn = ru_fma(cp, z.rn, ru_fma(cn, z.rh, ru_fma(s, z.ih, E)));
  r.ih = ru_fma(s, z.rh, ru_fma(cp, z.ih, ru_fma(cn, z.in, E)));
  r.in = ru_fma(s, z.rn, ru_fma(cp, z.in, ru_fma(cn, z.ih, E)));
  return r;
}

// Product of two stored roots as a point, with a bound valid for every pair:
// each computed component is within 2^-51 of the exact product of the stored
// points (two roundings of at most one ulp of a value of magnitude <= 1 + e),
// which is within e (|c1| + |s1| + |c2| + |s2|) + 2 e^2 <= 2 sqrt(2) e + 2 e^2
// of the true root; ep = pass_tw_bound(e) = 2^-50 + 3 e (rounded up) covers
// both for any e < 0.08.
__device__ __forceinline__ double pass_tw_bound(double e) {
  return ru_fma(3.0, e, 0x1p-50);
}
__device__ __forceinline__ double2 tw_point_product(double2 w1, double2 w2) {
  return make_double2(ru_fma(w1.x, w2.x, ru_nmul(w1.y, w2.y)), ru_fma(w1.x, w2.y, ru_mul(w1.y, w2.x)));
}

// Midpoint-radius form of the rectangular product (used for the pointwise
// products): an interval [-n, h] scaled by s (s = 1 or 1/2, exact) as a
// midpoint m and a radius r >= max(s h - m, m + s n), so m +- r encloses it
// whatever rounding m carries.
struct mrad {
  double m, r;
};
__device__ __forceinline__ mrad to_mrad(double n, double h, double s) {
  const double m = ru_mul(0.5 * s, ru_sub(h, n));
  return mrad{m, dmax(ru_fms(s, h, m), ru_fma(s, n, m))};
}
// (ar + i ai)(br + i bi) with every part a midpoint-radius interval:
//   Re = ar br - ai bi + d_re,  Im = ar bi + ai br + d_im,
//   |d_re| <= (|ar| + rar) rbr + rar |br| + (|ai| + rai) rbi + rai |bi|,
//   |d_im| <= (|ar| + rar) rbi + rar |bi| + (|ai| + rai) rbr + rai |br|
// (from (a + x)(b + y) - a b = a y + x b + x y); the midpoint products are
// bounded above and below by fused chains rounded up.  The result encloses the
// exact set of products of the paper's section 2.5, about 40 FP64 operations
// instead of 60 for the four-end-point form.
__device__ __forceinline__ ci ci_mul_mrad(mrad ar, mrad ai, mrad br, mrad bi) {
  const double t1 = ru_add_aa(ar.m, ar.r), t2 = ru_add_aa(ai.m, ai.r);
  const double dre = ru_fma(t1, br.r, ru_fma_ab(ar.r, br.m, ru_fma(t2, bi.r, ru_mul_ab(ai.r, bi.m))));
  const double dim = ru_fma(t1, bi.r, ru_fma_ab(ar.r, bi.m, ru_fma(t2, br.r, ru_mul_ab(ai.r, br.m))));
  ci o;
  o.rh = ru_add(ru_fma(ar.m, br.m, ru_nmul(ai.m, bi.m)), dre);
  o.rn = ru_add(ru_nfma(ar.m, br.m, ru_mul(ai.m, bi.m)), dre);
  o.ih = ru_add(ru_fma(ar.m, bi.m, ru_mul(ai.m, br.m)), dim);
  o.in = ru_add(ru_nfma(ar.m, bi.m, ru_nmul(ai.m, br.m)), dim);
  return o;
}
__device__ __forceinline__ ci ci_mul_fast(const ci &a, const ci &b) {
  return ci_mul_mrad(to_mrad(a.rn, a.rh, 1.0), to_mrad(a.in, a.ih, 1.0), to_mrad(b.rn, b.rh, 1.0),
                     to_mrad(b.in, b.ih, 1.0));
}

// Multiplication of every bound by 2^-k (exact unless it underflows; rounding
// up keeps both stored bounds valid either way).
__device__ __forceinline__ ci ci_scale(const ci &a, double p2) {
  return ci{ru_mul(a.rn, p2), ru_mul(a.rh, p2), ru_mul(a.in, p2), ru_mul(a.ih, p2)};
}

}  // namespace ssa
