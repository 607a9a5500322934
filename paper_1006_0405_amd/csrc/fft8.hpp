// Interval DFT of length M = 2^m (m >= 3) computed cooperatively by the M/8
// threads of a thread group, 8 elements per thread in registers, exchanges
// through LDS.
//
// The transform is the DFT of the paper (section 2.2) with omega = e^{+2 pi i/M}.
// It uses the Stockham (self-sorting) form of the Cooley-Tukey factorisation:
// one radix-2 or radix-4 stage when m is not a multiple of 3, then radix-8
// stages.  Stage s with radix R and Ns = product of the earlier radices: thread
// j takes v_r = x[j + r M/R], multiplies v_r by omega_{R Ns}^{r k} (k = j mod Ns),
// applies the length-R DFT and writes result q to y[(j - k) R + k + q Ns].  After
// the last stage (R Ns = M) result q of thread j is X[j + q M/8], already in the
// thread's registers, so input and output are both in natural order.
//
// Radix 8 needs two exchanges for M = 512 (radix 4 needs four), which halves
// the LDS traffic per element.  An exchange moves each element in two 16-byte
// words (a rectangle's real bounds, then its imaginary bounds; a disc's
// midpoint, then its radius), so the exchange buffer is M x 16 bytes.  The
// element type is a template parameter: rectangles (ci) and discs (md) provide
// the same operation names (e_add, e_tw, e_word0, ...).  When the group is one
// wavefront (M/8 <= 64) the exchanges need no workgroup barrier: LDS operations
// of one wavefront complete in order.
#pragma once
#include <type_traits>

#include "fft.hpp"

namespace ssa {

// Synchronisation of an exchange: a workgroup barrier, or within one wavefront
// only an ordering point for the compiler (the hardware keeps a wavefront's LDS
// operations in order).
template <bool WAVE> __device__ __forceinline__ void xsync() {
  if (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Multiplication by omega_8 = c (1 + i) and by omega_8^3 = c (-1 + i), with c a
// point within e of 1/sqrt(2):  (x + i y)(1 + i) = (x - y) + i (x + y) and
// (x + i y)(-1 + i) = -(x + y) + i (x - y); then c[u] is [c u.lo, c u.hi] widened
// by e |u|max.
__device__ __forceinline__ ci ci_mul_w8(const ci &z, double c, double e) {
  const double un = ru_add(z.rn, z.ih), uh = ru_add(z.rh, z.in);  // u = x - y
  const double wn = ru_add(z.rn, z.in), wh = ru_add(z.rh, z.ih);  // w = x + y
  const double Eu = ru_mul(e, dmax(un, uh)), Ew = ru_mul(e, dmax(wn, wh));
  return ci{ru_fma(c, un, Eu), ru_fma(c, uh, Eu), ru_fma(c, wn, Ew), ru_fma(c, wh, Ew)};
}
__device__ __forceinline__ ci ci_mul_w83(const ci &z, double c, double e) {
  const double un = ru_add(z.rn, z.ih), uh = ru_add(z.rh, z.in);  // u = x - y
  const double wn = ru_add(z.rn, z.in), wh = ru_add(z.rh, z.ih);  // w = x + y
  const double Eu = ru_mul(e, dmax(un, uh)), Ew = ru_mul(e, dmax(wn, wh));
  // re = -c w: bounds swap; im = c u
  return ci{ru_fma(c, wh, Ew), ru_fma(c, wn, Ew), ru_fma(c, un, Eu), ru_fma(c, uh, Eu)};
}

// Length-8 DFT with omega_8 = e^{+2 pi i/8}, as two length-4 DFTs:
// a_r = v_r + v_{r+4}, b_r = (v_r - v_{r+4}) omega_8^r (r < 4);
// y_{2m} = DFT4(a)_m, y_{2m+1} = DFT4(b)_m.  Only omega_8 and omega_8^3 are
// interval-inexact; omega_8^2 = i is a permutation.
// For discs omega_8 and omega_8^3 are rotations by the point (+-c8, c8).
__device__ __forceinline__ ci e_mul_w8(const ci &z, double c8, double e8) { return ci_mul_w8(z, c8, e8); }
__device__ __forceinline__ ci e_mul_w83(const ci &z, double c8, double e8) { return ci_mul_w83(z, c8, e8); }
__device__ __forceinline__ md e_mul_w8(const md &z, double c8, double e8) { return md_tw(z, c8, c8, e8); }
__device__ __forceinline__ md e_mul_w83(const md &z, double c8, double e8) { return md_tw(z, -c8, c8, e8); }
__device__ __forceinline__ pt e_mul_w8(const pt &z, double c8, double e8) { return e_tw(z, c8, c8, e8); }
__device__ __forceinline__ pt e_mul_w83(const pt &z, double c8, double e8) { return e_tw(z, -c8, c8, e8); }
__device__ __forceinline__ pf e_mul_w8(const pf &z, double c8, double e8) { return e_tw(z, c8, c8, e8); }
__device__ __forceinline__ pf e_mul_w83(const pf &z, double c8, double e8) { return e_tw(z, -c8, c8, e8); }

template <class E> __device__ __forceinline__ void radix8(E v[8], double c8, double e8) {
  E a[4], b[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    a[r] = e_add(v[r], v[r + 4]);
    b[r] = e_sub(v[r], v[r + 4]);
  }
  b[1] = e_mul_w8(b[1], c8, e8);
  b[2] = e_mul_i(b[2]);
  b[3] = e_mul_w83(b[3], c8, e8);
  radix4(a);
  radix4(b);
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    v[2 * m] = a[m];
    v[2 * m + 1] = b[m];
  }
}

// The length-8 DFT above for thin rectangles x_r + i y_r whose parts are small
// integers (the first stage of a transform of digits): their sums and
// differences are exact in any rounding, so they run on the points, and only
// the products by omega_8 and omega_8^3 (ci_mul_w8 / ci_mul_w83 of a thin
// value, u = x - y and w = x + y exact) form intervals.  The enclosures are
// those of radix8 on the thin rectangles (zero bounds may differ in sign).
// 76 FP64 operations instead of 120.
__device__ __forceinline__ ci thin_ci(double x, double y) { return ci{-x, x, -y, y}; }
__device__ __forceinline__ void radix8_thin(ci v[8], double c8, double e8) {
  double ax[4], ay[4], bx[4], by[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    ax[r] = ru_add(v[r].rh, v[r + 4].rh);
    ay[r] = ru_add(v[r].ih, v[r + 4].ih);
    bx[r] = ru_sub(v[r].rh, v[r + 4].rh);
    by[r] = ru_sub(v[r].ih, v[r + 4].ih);
  }
  // a: length-4 DFT on points (exact)
  const double Ax = ru_add(ax[0], ax[2]), Ay = ru_add(ay[0], ay[2]);
  const double Bx = ru_sub(ax[0], ax[2]), By = ru_sub(ay[0], ay[2]);
  const double Cx = ru_add(ax[1], ax[3]), Cy = ru_add(ay[1], ay[3]);
  const double Dx = ru_sub(ax[1], ax[3]), Dy = ru_sub(ay[1], ay[3]);
  // b1 omega_8, b3 omega_8^3
  const double u1 = ru_sub(bx[1], by[1]), w1 = ru_add(bx[1], by[1]);
  const double eu1 = ru_mul_ab(e8, u1), ew1 = ru_mul_ab(e8, w1);
  const ci B1{ru_nfma(c8, u1, eu1), ru_fma(c8, u1, eu1), ru_nfma(c8, w1, ew1), ru_fma(c8, w1, ew1)};
  const double u3 = ru_sub(bx[3], by[3]), w3 = ru_add(bx[3], by[3]);
  const double eu3 = ru_mul_ab(e8, u3), ew3 = ru_mul_ab(e8, w3);
  const ci B3{ru_fma(c8, w3, ew3), ru_nfma(c8, w3, ew3), ru_nfma(c8, u3, eu3), ru_fma(c8, u3, eu3)};
  // b: length-4 DFT of (b0, b1 omega_8, i b2, b3 omega_8^3)
  const double Px = ru_sub(bx[0], by[2]), Py = ru_add(by[0], bx[2]);  // b0 + i b2
  const double Qx = ru_add(bx[0], by[2]), Qy = ru_sub(by[0], bx[2]);  // b0 - i b2
  const ci C = ci_add(B1, B3), D = ci_mul_i(ci_sub(B1, B3));
  v[0] = thin_ci(ru_add(Ax, Cx), ru_add(Ay, Cy));
  v[4] = thin_ci(ru_sub(Ax, Cx), ru_sub(Ay, Cy));
  v[2] = thin_ci(ru_sub(Bx, Dy), ru_add(By, Dx));  // B + i D
  v[6] = thin_ci(ru_add(Bx, Dy), ru_sub(By, Dx));  // B - i D
  v[1] = ci_add(thin_ci(Px, Py), C);
  v[5] = ci_sub(thin_ci(Px, Py), C);
  v[3] = ci_add(thin_ci(Qx, Qy), D);
  v[7] = ci_sub(thin_ci(Qx, Qy), D);
}

// Half-element LDS buffers hold element i at h[lpad(i) * is]: one spare slot
// after every 8 elements, so that the stride-8 write patterns of the radix-8
// stages spread over the LDS banks.  A buffer for M elements needs
// lpad_size(M) slots.
__device__ __forceinline__ int lpad(int i) { return i + (i >> 3); }
__host__ __device__ constexpr size_t lpad_size(size_t m) { return m + (m >> 3); }

// Move the 8 values of this thread to positions wpos(q) and read back the
// values at rpos(r) = j + r M/8, in two 16-byte rounds.  Element i of the
// buffer lives at h[lpad(i) << lis].
template <bool WAVE, class E, class W>
__device__ __forceinline__ void exchange8(E v[8], int j, int M8, double2 *h, int lis, W wpos) {
  double2 t[8];
  xsync<WAVE>();
#pragma unroll
  for (int q = 0; q < 8; ++q) h[lpad(wpos(q)) << lis] = e_word0(v[q]);
  xsync<WAVE>();
#pragma unroll
  for (int r = 0; r < 8; ++r) t[r] = h[lpad(j + r * M8) << lis];
  if constexpr (e_traits<E>::words == 1) {
#pragma unroll
    for (int r = 0; r < 8; ++r) e_from_words(v[r], t[r], t[r]);
    return;
  }
  xsync<WAVE>();
#pragma unroll
  for (int q = 0; q < 8; ++q) h[lpad(wpos(q)) << lis] = e_word1(v[q]);
  xsync<WAVE>();
#pragma unroll
  for (int r = 0; r < 8; ++r) e_from_words(v[r], t[r], h[lpad(j + r * M8) << lis]);
}

// Forward interval DFT of the group's M = 2^LOGM elements (LOGM >= 3), a
// compile-time length so that the stage sequence and every index is fixed
// when the kernel is compiled.  `h` points at element 0 of this group's
// half-element exchange buffer; element i lives at h[lpad(i) << lis].  With
// WAVE the group must be exactly the lanes of (part of) one wavefront;
// otherwise every thread of the workgroup must call this with the same M.
template <int LOGM, bool WAVE, bool PF = false, class TT = twtab, class E = ci, bool LAZY = false,
          bool THIN = false>
__device__ __forceinline__ void fft8_group(E v[8], int j, double2 *h, int lis, const TT &T) {
  static_assert(LOGM >= 3, "length-8 groups at least");
  constexpr int M8 = 1 << (LOGM - 3);
  constexpr int FIRST = LOGM % 3;           // radix-2 (1) or radix-4 (2) first stage, or none (0)
  constexpr int NR8 = (LOGM - FIRST) / 3;   // radix-8 stages
  const double2 w8 = root(T, 3, 1);  // omega_8 from the table
  const double c8 = w8.x, e8 = T.e;  // |1/sqrt 2 - c8| <= e
  // PF: twiddles of the next radix-8 stage are loaded one stage ahead, so that
  // their latency overlaps the current stage's arithmetic and exchange (at the
  // cost of 28 more live registers); otherwise a stage's seven twiddles are
  // loaded together at its start, or with LAZY each right before its product
  // (the fewest live registers).
  double2 w[8];
  const auto load_tw = [&](int lns) {
    const int k = j & ((1 << lns) - 1);
#pragma unroll
    for (int r = 1; r < 8; ++r) w[r] = root(T, lns + 3, static_cast<uint32_t>(r * k));
  };
  if (PF && FIRST != 0) load_tw(FIRST);  // the first radix-8 stage has Ns = 2 or 4
  if (FIRST == 1) {
    // radix 2 (Ns = 1): this thread acts for positions jv = j + t M/8, t < 4,
    // pairs (x[jv], x[jv + M/2]) = (v_t, v_{t+4}); results to y[2 jv], y[2 jv + 1].
    E y[8];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      y[2 * t] = e_add(v[t], v[t + 4]);
      y[2 * t + 1] = e_sub(v[t], v[t + 4]);
    }
    exchange8<WAVE>(y, j, M8, h, lis, [&](int q) { return 2 * (j + (q >> 1) * M8) + (q & 1); });
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = y[r];
  } else if (FIRST == 2) {
    // radix 4 (Ns = 1): positions jv = j + t M/8, t < 2, elements
    // x[jv + s M/4] = v_{t + 2 s}; results to y[4 jv + q].
    E y[8];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      E u[4] = {v[t], v[t + 2], v[t + 4], v[t + 6]};
      radix4(u);
#pragma unroll
      for (int q = 0; q < 4; ++q) y[4 * t + q] = u[q];
    }
    exchange8<WAVE>(y, j, M8, h, lis, [&](int q) { return 4 * (j + (q >> 2) * M8) + (q & 3); });
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = y[r];
  }
#pragma unroll
  for (int st = 0; st < NR8; ++st) {
    const int logNs = FIRST + 3 * st;
    const int Ns = 1 << logNs;
    const int k = j & (Ns - 1);
    if (!PF && !LAZY && logNs > 0) load_tw(logNs);
    if (LAZY && logNs > 0) {
      // each twiddle loaded where it is used: fewer live registers
#pragma unroll
      for (int r = 1; r < 8; ++r) {
        const double2 wr = root(T, logNs + 3, static_cast<uint32_t>(r * k));
        v[r] = r <= 2 ? e_tw_q1(v[r], wr.x, wr.y, T.e)
             : r <= 4 ? e_tw_uh(v[r], wr.x, wr.y, T.e)
                      : e_tw(v[r], wr.x, wr.y, T.e);
      }
    } else if (logNs > 0) {
      // omega_{8 Ns}^{r k} with k < Ns has angle below r pi / 4: for r <= 2 the
      // root lies in the first quadrant, for r <= 4 in the upper half plane,
      // and so do the stored points (rounded to nearest from the same side)
#pragma unroll
      for (int r = 1; r < 8; ++r)
        v[r] = r <= 2 ? e_tw_q1(v[r], w[r].x, w[r].y, T.e)
             : r <= 4 ? e_tw_uh(v[r], w[r].x, w[r].y, T.e)
                      : e_tw(v[r], w[r].x, w[r].y, T.e);
    }
    if constexpr (THIN && FIRST == 0 && std::is_same<E, ci>::value) {
      if (st == 0) radix8_thin(v, c8, e8);  // THIN: the inputs are thin small integers
      else radix8(v, c8, e8);
    } else {
      radix8(v, c8, e8);
    }
    if (st + 1 == NR8) break;  // last stage: X[j + q M/8] = v[q]
    if (PF) load_tw(logNs + 3);
    const int base = ((j - k) << 3) + k;
    exchange8<WAVE>(v, j, M8, h, lis, [&](int q) { return base + q * Ns; });
  }
}

// Exchange of 4 values per thread (M = 4 M4 elements): write result q to
// position wpos(q), read back x[j + r M4]; two 16-byte rounds, padded slots.
template <bool WAVE, class E, class W>
__device__ __forceinline__ void exchange4(E v[4], int j, int M4, double2 *h, W wpos) {
  double2 t[4];
  xsync<WAVE>();
#pragma unroll
  for (int q = 0; q < 4; ++q) h[lpad(wpos(q))] = e_word0(v[q]);
  xsync<WAVE>();
#pragma unroll
  for (int r = 0; r < 4; ++r) t[r] = h[lpad(j + r * M4)];
  if constexpr (e_traits<E>::words == 1) {
#pragma unroll
    for (int r = 0; r < 4; ++r) e_from_words(v[r], t[r], t[r]);
    return;
  }
  xsync<WAVE>();
#pragma unroll
  for (int q = 0; q < 4; ++q) h[lpad(wpos(q))] = e_word1(v[q]);
  xsync<WAVE>();
#pragma unroll
  for (int r = 0; r < 4; ++r) e_from_words(v[r], t[r], h[lpad(j + r * M4)]);
}

// Forward interval DFT of M = 2^LOGM elements held 4 per thread by M/4
// threads: thread j holds x[j + r M/4], r < 4, and ends with X[j + q M/4].
// Stockham radix-4 stages (one radix-2 stage first when LOGM is odd), same
// conventions as fft8_group; the twiddles omega_{4 Ns}^{r k}, k < Ns, lie in
// the first quadrant for r = 1, the upper half plane for r = 2.  A stage's
// three twiddles are loaded before the exchange that precedes it, so that
// their latency overlaps the exchange.
template <int LOGM, bool WAVE, class TT = twtab, class E = ci>
__device__ __forceinline__ void fft4_group(E v[4], int j, double2 *h, const TT &T) {
  static_assert(LOGM >= 2, "length-4 groups at least");
  constexpr int M4 = 1 << (LOGM - 2);
  constexpr int FIRST = LOGM % 2;
  constexpr int NR4 = (LOGM - FIRST) / 2;
  double2 w1, w2, w3;
  const auto load_tw = [&](int lns) {
    const int kk = j & ((1 << lns) - 1);
    w1 = root(T, lns + 2, static_cast<uint32_t>(kk));
    w2 = root(T, lns + 2, static_cast<uint32_t>(2 * kk));
    w3 = root(T, lns + 2, static_cast<uint32_t>(3 * kk));
  };
  if (FIRST == 1) load_tw(1);
  if (FIRST == 1) {
    // radix 2 (Ns = 1): positions jv = j + t M/4 (t < 2) pair x[jv] = v_t with
    // x[jv + M/2] = v_{t+2}; results to y[2 jv], y[2 jv + 1]
    E y[4];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      y[2 * t] = e_add(v[t], v[t + 2]);
      y[2 * t + 1] = e_sub(v[t], v[t + 2]);
    }
    exchange4<WAVE>(y, j, M4, h, [&](int q) { return 2 * (j + (q >> 1) * M4) + (q & 1); });
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = y[r];
  }
#pragma unroll
  for (int st = 0; st < NR4; ++st) {
    const int logNs = FIRST + 2 * st;
    const int Ns = 1 << logNs;
    const int k = j & (Ns - 1);
    if (logNs > 0) {
      v[1] = e_tw_q1(v[1], w1.x, w1.y, T.e);
      v[2] = e_tw_uh(v[2], w2.x, w2.y, T.e);
      v[3] = e_tw(v[3], w3.x, w3.y, T.e);
    }
    radix4(v);
    if (st + 1 == NR4) break;  // X[j + q M/4] = v[q]
    load_tw(logNs + 2);
    const int base = ((j - k) << 2) + k;
    exchange4<WAVE>(v, j, M4, h, [&](int q) { return base + q * Ns; });
  }
}

}  // namespace ssa
