// Double-precision midpoint-radius (disc) complex intervals, the circular
// containment sets that the paper proposes as a variant of its rectangles
// (section 4), for the three-pass product path.
//
// An element is a disc {z : |z - m| <= r}, midpoint m = (re, im) and radius r,
// all FP64.  The kernels run with the FP64 rounding field of MODE at "toward
// +infinity" (enter_round_up), so
//   * a radius evaluated as a chain of additions and fused multiply-adds of
//     non-negative terms is an upper bound of its exact value;
//   * a midpoint computed by one rounded operation, y = RU(x), is within one
//     ulp of x: |y - x| <= 2^-52 |y| when y is normal, and < 2^-1074 when y is
//     subnormal (a subnormal sum or difference is exact, so only products and
//     fused multiply-adds add the absolute term).
// Every operation adds these rounding terms to the radius.  A rotation by a
// root of unity does not enlarge a disc (|w| = 1), where the rectangular hull
// of a rotated rectangle grows by |cos| + |sin|.
#pragma once
#include "ia.hpp"

namespace ssa {

struct md {
  double re, im, r;
};

static constexpr double MD_U = 0x1p-52;      // relative bound of one directed rounding
static constexpr double MD_ETA = 0x1p-1074;  // absolute bound of a subnormal product's rounding

__device__ __forceinline__ md md_add(const md &a, const md &b) {
  md c;
  c.re = ru_add(a.re, b.re);
  c.im = ru_add(a.im, b.im);
  c.r = ru_fma_ab(MD_U, c.re, ru_fma_ab(MD_U, c.im, ru_add(a.r, b.r)));
  return c;
}
__device__ __forceinline__ md md_sub(const md &a, const md &b) {
  md c;
  c.re = ru_sub(a.re, b.re);
  c.im = ru_sub(a.im, b.im);
  c.r = ru_fma_ab(MD_U, c.re, ru_fma_ab(MD_U, c.im, ru_add(a.r, b.r)));
  return c;
}
// Exact: i z, -i z, conj z, 2^k z (scaling by a power of two is exact unless
// the midpoint underflows; MD_ETA in the radius covers that case).
__device__ __forceinline__ md md_mul_i(const md &a) { return md{-a.im, a.re, a.r}; }
__device__ __forceinline__ md md_mul_negi(const md &a) { return md{a.im, -a.re, a.r}; }
__device__ __forceinline__ md md_conj(const md &a) { return md{a.re, -a.im, a.r}; }
__device__ __forceinline__ md md_scale(const md &a, double p2) {
  return md{ru_mul(a.re, p2), ru_mul(a.im, p2), ru_fma(a.r, p2, 2.0 * MD_ETA)};
}

// w a for a point w = (c, s) within e of a root of unity w* in each component
// (|w - w*| <= sqrt(2) e < 1.5 e, |w*| = 1):
//   |m' - w* a*| <= |m' - w m| + |w - w*| |m| + |w*| |m - a*|
//               <= rounding + 1.5 e (|re| + |im|) + r.
// m' = (RU(c re - p), RU(s re + q)) with p = RU(s im), q = RU(c im): four
// roundings, each within 2^-52 of its result plus MD_ETA, and the four results
// sum to at most (1 + 2^-52)^2 (|c| + |s|) (|re| + 2 |im|) + 6 MD_ETA with
// |c| + |s| <= sqrt(2) (1 + 1.5 e): below 2.9 (|re| + |im|) for e < 2^-20.  So
//   r' = r + (1.5 e + 2.9 2^-52) (|re| + |im|) + 8 MD_ETA,
// three operations instead of one per rounding.
__device__ __forceinline__ md md_tw(const md &a, double c, double s, double e) {
  const double p = ru_mul(s, a.im), q = ru_mul(c, a.im);
  md z;
  z.re = ru_fms(c, a.re, p);
  z.im = ru_fma(s, a.re, q);
  const double k = ru_fma(1.5, e, 2.9 * MD_U);
  z.r = ru_fma_ab(k, a.re, ru_fma_ab(k, a.im, ru_add(a.r, 8.0 * MD_ETA)));
  return z;
}

// Product of two discs: m' = (a.re b.re - a.im b.im, a.re b.im + a.im b.re)
// with four roundings (p1 = RU(a.im b.im), p2 = RU(a.im b.re)), and
//   |a* b* - m_a m_b| <= |m_a| r_b + r_a |m_b| + r_a r_b,
// |m| <= |re| + |im|.  The four rounded results sum to at most
// (1 + 2^-52)^2 2 ma mb' + 4 MD_ETA (ma = |a.re| + |a.im|, mb' = |b.re| + |b.im|),
// so the roundings add at most 2.0001 2^-52 ma mb' + 5 MD_ETA:
//   r' = ma (r_b + 2.0001 2^-52 mb') + r_a (mb' + r_b) + 8 MD_ETA.
__device__ __forceinline__ md md_mul(const md &a, const md &b) {
  const double p1 = ru_mul(a.im, b.im), p2 = ru_mul(a.im, b.re);
  md z;
  z.re = ru_fms(a.re, b.re, p1);
  z.im = ru_fma(a.re, b.im, p2);
  const double ma = ru_add_aa(a.re, dabs(a.im));  // |a.re| + |a.im|
  const double mb = ru_add_aa(b.re, dabs(b.im));  // |b.re| + |b.im|
  const double t = ru_fma(2.0001 * MD_U, mb, b.r);
  z.r = ru_fma(ma, t, ru_fma(a.r, ru_add(mb, b.r), 8.0 * MD_ETA));
  return z;
}

// Real-part and imaginary-part enclosures in the kernels' negated-lower form:
// [re - r, re + r] as (RU(r - re), RU(re + r)).
__device__ __forceinline__ double md_re_n(const md &a) { return ru_sub(a.r, a.re); }
__device__ __forceinline__ double md_re_h(const md &a) { return ru_add(a.re, a.r); }
__device__ __forceinline__ double md_im_n(const md &a) { return ru_sub(a.r, a.im); }
__device__ __forceinline__ double md_im_h(const md &a) { return ru_add(a.im, a.r); }

// ---- The element interface the generic DFT and the kernels use ------------
// Rectangles (ci) and discs (md) provide the same set of names, so one source
// serves both element types; for ci every name is the rectangular operation.

__device__ __forceinline__ ci e_add(const ci &a, const ci &b) { return ci_add(a, b); }
__device__ __forceinline__ ci e_sub(const ci &a, const ci &b) { return ci_sub(a, b); }
__device__ __forceinline__ ci e_mul_i(const ci &a) { return ci_mul_i(a); }
__device__ __forceinline__ ci e_mul_negi(const ci &a) { return ci_mul_negi(a); }
__device__ __forceinline__ ci e_conj(const ci &a) { return ci_conj(a); }
__device__ __forceinline__ ci e_scale(const ci &a, double p2) { return ci_scale(a, p2); }
__device__ __forceinline__ ci e_tw(const ci &a, double c, double s, double e) { return ci_twiddle(a, c, s, e); }
__device__ __forceinline__ ci e_tw_q1(const ci &a, double c, double s, double e) {
  return ci_twiddle_q1(a, c, s, e);
}
__device__ __forceinline__ ci e_tw_uh(const ci &a, double c, double s, double e) {
  return ci_twiddle_uh(a, c, s, e);
}
// the two 16-byte words of an element for an LDS exchange, and back
__device__ __forceinline__ double2 e_word0(const ci &a) { return make_double2(a.rn, a.rh); }
__device__ __forceinline__ double2 e_word1(const ci &a) { return make_double2(a.in, a.ih); }
__device__ __forceinline__ void e_from_words(ci &a, double2 w0, double2 w1) { a = ci{w0.x, w0.y, w1.x, w1.y}; }

__device__ __forceinline__ md e_add(const md &a, const md &b) { return md_add(a, b); }
__device__ __forceinline__ md e_sub(const md &a, const md &b) { return md_sub(a, b); }
__device__ __forceinline__ md e_mul_i(const md &a) { return md_mul_i(a); }
__device__ __forceinline__ md e_mul_negi(const md &a) { return md_mul_negi(a); }
__device__ __forceinline__ md e_conj(const md &a) { return md_conj(a); }
__device__ __forceinline__ md e_scale(const md &a, double p2) { return md_scale(a, p2); }
__device__ __forceinline__ md e_tw(const md &a, double c, double s, double e) { return md_tw(a, c, s, e); }
__device__ __forceinline__ md e_tw_q1(const md &a, double c, double s, double e) { return md_tw(a, c, s, e); }
__device__ __forceinline__ md e_tw_uh(const md &a, double c, double s, double e) { return md_tw(a, c, s, e); }
__device__ __forceinline__ double2 e_word0(const md &a) { return make_double2(a.re, a.im); }
__device__ __forceinline__ double2 e_word1(const md &a) { return make_double2(a.r, 0.0); }
__device__ __forceinline__ void e_from_words(md &a, double2 w0, double2 w1) { a = md{w0.x, w0.y, w1.x}; }

// ---- Point complex numbers (a non-rigorous baseline) ----------------------
// The same transforms with plain double complex values, round to nearest (the
// kernels of this type leave MODE at its default): the naive method whose
// cost the interval arithmetic is compared against.  Nothing is certified.
struct pt {
  double re, im;
};
__device__ __forceinline__ pt e_add(const pt &a, const pt &b) { return pt{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ pt e_sub(const pt &a, const pt &b) { return pt{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ pt e_mul_i(const pt &a) { return pt{-a.im, a.re}; }
__device__ __forceinline__ pt e_mul_negi(const pt &a) { return pt{a.im, -a.re}; }
__device__ __forceinline__ pt e_conj(const pt &a) { return pt{a.re, -a.im}; }
__device__ __forceinline__ pt e_scale(const pt &a, double p2) { return pt{a.re * p2, a.im * p2}; }
__device__ __forceinline__ pt e_tw(const pt &a, double c, double s, double) {
  return pt{c * a.re - s * a.im, s * a.re + c * a.im};
}
__device__ __forceinline__ pt e_tw_q1(const pt &a, double c, double s, double e) { return e_tw(a, c, s, e); }
__device__ __forceinline__ pt e_tw_uh(const pt &a, double c, double s, double e) { return e_tw(a, c, s, e); }
__device__ __forceinline__ double2 e_word0(const pt &a) { return make_double2(a.re, a.im); }
__device__ __forceinline__ double2 e_word1(const pt &) { return make_double2(0.0, 0.0); }
__device__ __forceinline__ void e_from_words(pt &a, double2 w0, double2) { a = pt{w0.x, w0.y}; }

// ---- Single-precision point complex numbers (the naive FP32 baseline) ------
// The paper's section 1 observation concerns this arithmetic: a naive
// single-precision transform is usually right and sometimes wrong already at
// 120 base-256 digits.  Plain float complex values, round to nearest, the
// double twiddles rounded to float; an exchange moves the pair as one 8-byte
// word (the low half of a 16-byte slot).  Nothing is certified.
struct pf {
  float re, im;
};
__device__ __forceinline__ pf e_add(const pf &a, const pf &b) { return pf{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ pf e_sub(const pf &a, const pf &b) { return pf{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ pf e_mul_i(const pf &a) { return pf{-a.im, a.re}; }
__device__ __forceinline__ pf e_mul_negi(const pf &a) { return pf{a.im, -a.re}; }
__device__ __forceinline__ pf e_conj(const pf &a) { return pf{a.re, -a.im}; }
__device__ __forceinline__ pf e_scale(const pf &a, double p2) {
  const float f = static_cast<float>(p2);  // a power of two: exact
  return pf{a.re * f, a.im * f};
}
__device__ __forceinline__ pf e_tw(const pf &a, double c, double s, double) {
  const float cf = static_cast<float>(c), sf = static_cast<float>(s);
  return pf{cf * a.re - sf * a.im, sf * a.re + cf * a.im};
}
__device__ __forceinline__ pf e_tw_q1(const pf &a, double c, double s, double e) { return e_tw(a, c, s, e); }
__device__ __forceinline__ pf e_tw_uh(const pf &a, double c, double s, double e) { return e_tw(a, c, s, e); }
__device__ __forceinline__ double2 e_word0(const pf &a) {
  return make_double2(__builtin_bit_cast(double, make_float2(a.re, a.im)), 0.0);
}
__device__ __forceinline__ double2 e_word1(const pf &) { return make_double2(0.0, 0.0); }
__device__ __forceinline__ void e_from_words(pf &a, double2 w0, double2) {
  const float2 f = __builtin_bit_cast(float2, w0.x);
  a = pf{f.x, f.y};
}

// Per element type: whether it is an enclosure (rigorous) and how many 16-byte
// words an LDS exchange moves.
template <class E> struct e_traits {
  static constexpr bool rigorous = true;
  static constexpr int words = 2;
};
template <> struct e_traits<pt> {
  static constexpr bool rigorous = false;
  static constexpr int words = 1;
};
template <> struct e_traits<pf> {
  static constexpr bool rigorous = false;
  static constexpr int words = 1;
};

}  // namespace ssa
