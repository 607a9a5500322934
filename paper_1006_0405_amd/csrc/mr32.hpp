// Single-precision midpoint-radius (disc) complex intervals and their radix-8
// DFT, for the reduced-precision first attempt at a product.
//
// An element is a disc {z : |z - m| <= r} with midpoint m = (re, im) and radius
// r, all in FP32 with round-to-nearest (the FP32 rounding field of MODE is left
// at nearest-even).  Every operation computes the midpoint in FP32 and grows the
// radius by a rigorous bound of what the midpoint computation lost:
//   * for a round-to-nearest result y = fl(x), |y - x| <= U |y| + ETA with
//     U = 2^-24 and ETA = 2^-126 covering underflow and flushed subnormals;
//   * the radius is itself evaluated in round-to-nearest and then multiplied by
//     (1 + 8 U), which dominates the rounding of the few non-negative terms it
//     adds.
// Rotations by roots of unity do not enlarge a disc (unlike a rectangle), which
// is why this form is used for the single-precision attempt (circular
// containment sets, paper section 4).  The twiddles are the double-precision
// table rounded to FP32, with a bound E32 on each component's distance to the
// true root.
#pragma once
#include "fft8.hpp"

namespace ssa {

struct mr {
  float re, im, r;
};

static constexpr float MR_U = 5.9604644775390625e-08f;    // 2^-24
static constexpr float MR_ETA = 1.1754943508222875e-38f;  // 2^-126
static constexpr float MR_UP = 1.0f + 8.0f * MR_U;        // exact: 1 + 2^-21
// |(float)c - cos| <= |(float)c - c| + |c - cos| <= 2^-24 + e64 for |c| <= 1 in
// any rounding direction of the conversion (one FP32 ulp below 1 is 2^-24),
// and e64 < 2^-47: bounded by the next float above 2^-24.
static constexpr float MR_E32 = 5.9604651880817983e-08f;  // 2^-24 (1 + 2^-23)

__device__ __forceinline__ float fabs_(float x) { return __builtin_fabsf(x); }

__device__ __forceinline__ mr mr_add(const mr &a, const mr &b) {
  mr c;
  c.re = a.re + b.re;
  c.im = a.im + b.im;
  c.r = (a.r + b.r + MR_U * (fabs_(c.re) + fabs_(c.im)) + 2.0f * MR_ETA) * MR_UP;
  return c;
}
__device__ __forceinline__ mr mr_sub(const mr &a, const mr &b) {
  mr c;
  c.re = a.re - b.re;
  c.im = a.im - b.im;
  c.r = (a.r + b.r + MR_U * (fabs_(c.re) + fabs_(c.im)) + 2.0f * MR_ETA) * MR_UP;
  return c;
}
__device__ __forceinline__ mr mr_mul_i(const mr &a) { return mr{-a.im, a.re, a.r}; }

// w a with w = (c, s) within e of a root of unity (|w_true| = 1):
// |m - w_true a_true| <= (rounding of m) + |w_m| r_a + |w_m - w_true| (|a_m| + r_a),
// |w_m| <= 1 + 2e, |w_m - w_true| <= sqrt(2) e < 1.5 e, |a_m| <= |re| + |im|.
__device__ __forceinline__ mr mr_tw(const mr &a, float c, float s, float e) {
  const float p = s * a.im, q = c * a.im;
  mr z;
  z.re = __builtin_fmaf(c, a.re, -p);
  z.im = __builtin_fmaf(s, a.re, q);
  const float round = MR_U * (fabs_(z.re) + fabs_(z.im) + fabs_(p) + fabs_(q)) + 4.0f * MR_ETA;
  z.r = ((1.0f + 2.0f * e) * a.r + 1.5f * e * (fabs_(a.re) + fabs_(a.im) + a.r) + round) * MR_UP;
  return z;
}

__device__ __forceinline__ mr mr_tw_tab(const mr &a, const double2 w) {
  return mr_tw(a, static_cast<float>(w.x), static_cast<float>(w.y), MR_E32);
}

__device__ __forceinline__ void mr_radix4(mr v[4]) {
  const mr a = mr_add(v[0], v[2]), b = mr_sub(v[0], v[2]);
  const mr c = mr_add(v[1], v[3]), d = mr_sub(v[1], v[3]);
  const mr id = mr_mul_i(d);
  v[0] = mr_add(a, c);
  v[2] = mr_sub(a, c);
  v[1] = mr_add(b, id);
  v[3] = mr_sub(b, id);
}

// Length-8 DFT (omega_8 = e^{+2 pi i/8}) as two length-4 DFTs, see radix8.
__device__ __forceinline__ void mr_radix8(mr v[8], float c8) {
  mr a[4], b[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    a[r] = mr_add(v[r], v[r + 4]);
    b[r] = mr_sub(v[r], v[r + 4]);
  }
  b[1] = mr_tw(b[1], c8, c8, MR_E32);   // (1 + i)/sqrt 2
  b[2] = mr_mul_i(b[2]);
  b[3] = mr_tw(b[3], -c8, c8, MR_E32);  // (-1 + i)/sqrt 2
  mr_radix4(a);
  mr_radix4(b);
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    v[2 * m] = a[m];
    v[2 * m + 1] = b[m];
  }
}

// Exchange: one 16-byte slot (re, im, r, unused) per element.
template <bool WAVE, class W>
__device__ __forceinline__ void mr_exchange8(mr v[8], int j, int M8, float4 *h, W wpos) {
  xsync<WAVE>();
#pragma unroll
  for (int q = 0; q < 8; ++q) h[lpad(wpos(q))] = make_float4(v[q].re, v[q].im, v[q].r, 0.0f);
  xsync<WAVE>();
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const float4 t = h[lpad(j + r * M8)];
    v[r] = mr{t.x, t.y, t.z};
  }
}

// Forward DFT of M = 2^LOGM disc intervals, same Stockham schedule as
// fft8_group; h holds lpad_size(M) slots of 16 bytes.
template <int LOGM, bool WAVE>
__device__ __forceinline__ void mr_fft8_group(mr v[8], int j, float4 *h, const twtab &T) {
  constexpr int M8 = 1 << (LOGM - 3);
  constexpr int FIRST = LOGM % 3;
  constexpr int NR8 = (LOGM - FIRST) / 3;
  const float c8 = static_cast<float>(root(T, 3, 1).x);
  if (FIRST == 1) {
    mr y[8];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      y[2 * t] = mr_add(v[t], v[t + 4]);
      y[2 * t + 1] = mr_sub(v[t], v[t + 4]);
    }
    mr_exchange8<WAVE>(y, j, M8, h, [&](int q) { return 2 * (j + (q >> 1) * M8) + (q & 1); });
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = y[r];
  } else if (FIRST == 2) {
    mr y[8];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      mr u[4] = {v[t], v[t + 2], v[t + 4], v[t + 6]};
      mr_radix4(u);
#pragma unroll
      for (int q = 0; q < 4; ++q) y[4 * t + q] = u[q];
    }
    mr_exchange8<WAVE>(y, j, M8, h, [&](int q) { return 4 * (j + (q >> 2) * M8) + (q & 3); });
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = y[r];
  }
#pragma unroll
  for (int st = 0; st < NR8; ++st) {
    const int logNs = FIRST + 3 * st;
    const int Ns = 1 << logNs;
    const int k = j & (Ns - 1);
    if (logNs > 0) {
#pragma unroll
      for (int r = 1; r < 8; ++r) v[r] = mr_tw_tab(v[r], root(T, logNs + 3, static_cast<uint32_t>(r * k)));
    }
    mr_radix8(v, c8);
    if (st + 1 == NR8) break;
    const int base = ((j - k) << 3) + k;
    mr_exchange8<WAVE>(v, j, M8, h, [&](int q) { return base + q * Ns; });
  }
}

// The disc as a double rectangle: re in [m.re - r, m.re + r], im likewise,
// bounds rounded up in the negated-lower form (conversions float -> double are
// exact).
__device__ __forceinline__ ci mr_to_ci(const mr &a) {
  const double re = static_cast<double>(a.re), im = static_cast<double>(a.im);
  const double r = static_cast<double>(a.r);
  return ci{ru_add(-re, r), ru_add(re, r), ru_add(-im, r), ru_add(im, r)};
}

}  // namespace ssa
