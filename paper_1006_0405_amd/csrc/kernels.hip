// Kernels of the rigorous interval Schoenhage-Strassen product on gfx950.
//
// Fast convolution (paper section 2.3) over rectangular complex intervals
// (section 2.5), certification (section 1: the unique integer in each
// enclosure, else an error) and carries (section 2.4).
//
// Two shapes of the same computation:
//  * N <= 2^12: one workgroup per product, everything in LDS (k_small).
//  * larger N = N1 * N2: three passes of the four-step factorisation
//      X[k1 + N1 k2] = sum_n2 omega_N2^{n2 k2} omega_N^{n2 k1} sum_n1 x[N2 n1 + n2] omega_N1^{n1 k1}
//    k_col_fwd : length-N1 column DFTs of both operands, twiddle omega_N^{n2 k1},
//                rows k1 stored contiguously;
//    k_row     : per row k1 the length-N2 DFTs of both operands, the pointwise
//                product, and the first half of the inverse -- the spectrum never
//                leaves the chip.  The coefficients are real, so the inverse is
//                the half-length one of x_{2m} + i x_{2m+1} (half_inverse_input):
//                the row DFT of the conjugate is N2/2 long and only N2/2 values
//                per row go back to memory;
//    k_col_inv : length-N1 inverse column DFTs over the N2/2 remaining columns,
//                the 1/N scale, certification of both parts;
//    k_carry   : carries as a generate/propagate scan with decoupled look-back.
// The inverse DFT is computed as conj(DFT(conj(.)))/N, so a single forward
// interval DFT serves every transform; conjugation is exact.  The packed-path
// kernels take the element type as a template parameter: rectangles (ci, the
// paper's section 2.5) or FP64 discs (md, its section 4 variant).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "fft8.hpp"
#include "mr32.hpp"
#include "internal.hpp"

namespace ssa {

// ---------------------------------------------------------------------------
// Digits (section 2: little-endian base-b vectors); base 16 splits each byte
// into (low nibble, high nibble).

// Digit i of an operand with nd >= 1 digits (0 past the end), in two steps so
// that every load of a thread is issued before the first wait: load_digit
// reads the byte holding digit i (clamped into the operand, no branch) and
// digit_value extracts the digit and discards it past the end.
__device__ __forceinline__ uint32_t load_digit(const uint8_t *p, uint32_t nd, uint32_t i, int bits) {
  const uint32_t ic = i < nd ? i : nd - 1u;
  return gload(p + (ic >> (bits == 4 ? 1 : 0)));
}
__device__ __forceinline__ double digit_value(uint32_t raw, uint32_t nd, uint32_t i, int bits) {
  const uint32_t half = bits == 4 ? 1u : 0u;
  const uint32_t x = (raw >> ((i & half) << 2)) & (half ? 15u : 255u);
  return static_cast<double>(i < nd ? x : 0u);
}

// ---------------------------------------------------------------------------
// Certification of one enclosure.

struct cert_acc {
  double rad;
  uint32_t too_wide, internal, half;
};

static constexpr double TWO52 = 4503599627370496.0;

// For i < L the real enclosure [lo, hi] = [-n, h] of coefficient i must hold
// exactly one integer: ceil(lo) == floor(hi) (ceil(lo) = -floor(n)).  Several
// integers: too wide.  No integer, a negative one, or (im0 false) an imaginary
// part that excludes 0: impossible for a rigorous enclosure, counted as
// internal.  The padded tail i >= L must contain 0.
__device__ __forceinline__ unsigned long long certify_re(double n, double h, bool im0, uint32_t i,
                                                         uint32_t L, int mode, cert_acc &acc) {
  if (i >= L) {
    if (!(n >= 0.0 && h >= 0.0 && im0)) acc.internal++;
    return 0ull;
  }
  if (mode >= CERT_CORRUPT_BASE && i == static_cast<uint32_t>(mode - CERT_CORRUPT_BASE))
    h = ru_add(h, -1.0);  // test hook: this enclosure no longer holds its integer
  const double rad = ru_mul(ru_add(n, h), 0.5);
  acc.rad = rad > acc.rad ? rad : acc.rad;
  const double m = -dfloor(n);  // ceil(lo)
  const double M = dfloor(h);   // floor(hi)
  const double h_lo = -dfloor(ru_add(n, 0.5));  // ceil(lo - 1/2)
  const double h_hi = dfloor(ru_add(h, -0.5));  // floor(hi - 1/2)
  const bool half = h_lo <= h_hi;
  if (half) acc.half++;
  if (!(m <= M) || !im0) {
    acc.internal++;
    return 0ull;
  }
  if (m < M || (mode == CERT_HALF_INTEGER && half) || mode == CERT_FORCE_TOO_WIDE) {
    acc.too_wide++;
    return 0ull;
  }
  if (!(m >= 0.0 && m < TWO52)) {
    acc.internal++;
    return 0ull;
  }
  // m is an integer in [0, 2^52): m + 2^52 is exact and its low mantissa bits are m.
  const double t = ru_add(m, TWO52);
  return static_cast<unsigned long long>(__double_as_longlong(t)) - 0x4330000000000000ull;
}
// A complex enclosure of a real coefficient: the imaginary part must contain 0.
__device__ __forceinline__ unsigned long long certify(const ci &z, uint32_t i, uint32_t L,
                                                      int mode, cert_acc &acc) {
  return certify_re(z.rn, z.rh, z.in >= 0.0 && z.ih >= 0.0, i, L, mode, acc);
}

__device__ __forceinline__ void dbg_store(double *dbg, uint32_t i, const ci &z) {
  double2 *p = reinterpret_cast<double2 *>(dbg + 4 * static_cast<size_t>(i));
  p[0] = make_double2(-z.rn, z.rh);
  p[1] = make_double2(-z.in, z.ih);
}

// Block-wide reduction of the certification counters into LDS words, then
// (optionally) one atomic per block into the product's statistics.
struct cert_shared {
  unsigned long long rad_bits;
  unsigned long long half;
  unsigned int too_wide, internal;
};

__device__ __forceinline__ void cert_reduce(cert_shared &sh, const cert_acc &acc) {
  // acc.rad >= 0: the bit pattern orders like the value
  unsigned long long rb = static_cast<unsigned long long>(__double_as_longlong(acc.rad));
  uint32_t tw = acc.too_wide, in = acc.internal, hf = acc.half;
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(rb, off);
    rb = o > rb ? o : rb;
    tw += __shfl_xor(tw, off);
    in += __shfl_xor(in, off);
    hf += __shfl_xor(hf, off);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(&sh.rad_bits, rb);
    if (hf) atomicAdd(&sh.half, static_cast<unsigned long long>(hf));
    if (tw) atomicAdd(&sh.too_wide, tw);
    if (in) atomicAdd(&sh.internal, in);
  }
}

// ---------------------------------------------------------------------------
// Carries.
//
// The product is z = sum_i c_i 256^i with c_i < 2^48 (base-16 coefficients are
// first paired: C_j = c_{2j} + 16 c_{2j+1}).  Split every coefficient into
// bytes: s_p = sum_{t<6} byte_t(C_{p-t}) <= 6 * 255, then
// u_p = (s_p mod 256) + floor(s_{p-1} / 256) <= 260, so that z = sum u_p 256^p
// and the carry into every position is 0 or 1.  Position p generates a carry
// when u_p >= 256 and propagates one when u_p == 255; the carries are the
// prefix of these (generate, propagate) pairs.  Within a wavefront the prefix
// is an integer addition over the lane masks: with x = g | p, the carry into
// lane l is bit l of (x + g + cin) ^ x ^ g.

template <class F>
__device__ __forceinline__ uint32_t s_at(F C, long long p) {
  uint32_t s = 0;
#pragma unroll
  for (int t = 0; t < 6; ++t) {
    const unsigned long long v = C(p - t);
    s += static_cast<uint32_t>((v >> (8 * t)) & 255ull);
  }
  return s;
}

// One tile of positions [p0, p0 + waves * CHUNKS * 64).  Wave w owns CHUNKS
// consecutive chunks of 64 positions, one position per lane, so every load and
// store is lane-contiguous.  Per chunk the (generate, propagate) masks come
// from two ballots; a chunk's carry-out for carry-in c is G | (P & c) with
// G = carry out of x + g and P = "all lanes propagate".  `tile_cin(G, P)` is
// called by thread 0 with the tile's aggregate and returns the tile's carry-in.
template <int CHUNKS, class F, class TC>
__device__ __forceinline__ void carry_block(F C, long long p0, uint32_t nout, uint8_t *out,
                                            bool zero, TC tile_cin, uint32_t *sh_waves) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6, nwaves = blockDim.x >> 6;
  const long long wbase = p0 + static_cast<long long>(wave) * (CHUNKS * 64);
  uint32_t u[CHUNKS];
  unsigned long long gm[CHUNKS], pm[CHUNKS];
  uint32_t s_last = s_at(C, wbase - 1);  // s at the position before this wave's first
#pragma unroll
  for (int k = 0; k < CHUNKS; ++k) {
    const long long p = wbase + k * 64 + lane;
    const uint32_t s = s_at(C, p);
    uint32_t sp = __shfl_up(s, 1);
    if (lane == 0) sp = s_last;
    s_last = __shfl(s, 63);
    u[k] = (s & 255u) + (sp >> 8);
    gm[k] = __ballot(u[k] >= 256u);
    pm[k] = __ballot(u[k] == 255u);
  }
  uint32_t WG = 0, WP = 1;
#pragma unroll
  for (int k = 0; k < CHUNKS; ++k) {
    const unsigned long long x = gm[k] | pm[k];
    const uint32_t cg = (x + gm[k]) < x ? 1u : 0u;
    const uint32_t cp = pm[k] == ~0ull ? 1u : 0u;
    WG = cg | (cp & WG);
    WP &= cp;
  }
  if (lane == 0) sh_waves[wave] = (WG << 1) | WP;
  __syncthreads();
  if (tid == 0) {
    uint32_t TG = 0, TP = 1;
    for (int w = 0; w < nwaves; ++w) {
      const uint32_t a = sh_waves[w];
      TG = ((a >> 1) & 1u) | ((a & 1u) & TG);
      TP &= a & 1u;
    }
    uint32_t cin = zero ? 0u : tile_cin(TG, TP);
    for (int w = 0; w < nwaves; ++w) {
      const uint32_t a = sh_waves[w];
      sh_waves[w] = (a & 3u) | (cin << 2);
      cin = ((a >> 1) & 1u) | ((a & 1u) & cin);
    }
  }
  __syncthreads();
  uint32_t cin = (sh_waves[wave] >> 2) & 1u;
#pragma unroll
  for (int k = 0; k < CHUNKS; ++k) {
    const unsigned long long x = gm[k] | pm[k];
    const unsigned long long carries = (x + gm[k] + cin) ^ x ^ gm[k];
    const uint32_t cy = static_cast<uint32_t>((carries >> lane) & 1ull);
    const long long p = wbase + k * 64 + lane;
    if (p < static_cast<long long>(nout))
      gstore(out + p, zero ? static_cast<uint8_t>(0) : static_cast<uint8_t>(u[k] + cy));
    const uint32_t cg = (x + gm[k]) < x ? 1u : 0u;
    const uint32_t cp = pm[k] == ~0ull ? 1u : 0u;
    cin = cg | (cp & cin);
  }
}

// Both operands' transforms from one transform of z = a + i b (a, b real):
// A_k = (Z_k + conj Z_{-k}) / 2 and B_k = (Z_k - conj Z_{-k}) / (2i); the
// returned value encloses C_k = A_k B_k.  W = conj(Z_{-k}).  Conjugation,
// multiplication by -i and by 1/2 are exact, so this is as rigorous as the
// interval sum, difference and product it uses.
__device__ __forceinline__ ci separated_product(const ci &Z, const ci &W) {
  const ci S = ci_add(Z, W), D = ci_sub(Z, W);
  // A = S / 2;  B = -i D / 2, so Re B = Im D / 2 and Im B = -Re D / 2
  return ci_mul_mrad(to_mrad(S.rn, S.rh, 0.5), to_mrad(S.in, S.ih, 0.5),
                     to_mrad(D.in, D.ih, 0.5), to_mrad(D.rh, D.rn, 0.5));
}

// The same for discs: S = Z + W and D = Z - W, A = S/2 and B = -i D/2 (exact
// scalings and a permutation), C = A B.
__device__ __forceinline__ md separated_product(const md &Z, const md &W) {
  const md S = md_add(Z, W), D = md_sub(Z, W);
  return md_mul(md{0.5 * S.re, 0.5 * S.im, 0.5 * S.r}, md{0.5 * D.im, -0.5 * D.re, 0.5 * D.r});
}

// FP64 rounding for an element type: toward +infinity for the enclosures, the
// default (to nearest) for the point baseline.
template <class E> __device__ __forceinline__ uint32_t enter_mode() {
  if constexpr (e_traits<E>::rigorous) return enter_round_up();
  return 0u;
}

// The point baseline's coefficient: the nearest integer, no certificate; the
// distance to it is reported in place of a radius.
__device__ __forceinline__ unsigned long long naive_round(double x, uint32_t i, uint32_t L,
                                                          cert_acc &acc) {
  if (i >= L) return 0ull;
  const double m = __builtin_rint(x);
  const double d = __builtin_fabs(x - m);
  acc.rad = d > acc.rad ? d : acc.rad;
  return m > 0.0 ? static_cast<unsigned long long>(m) : 0ull;
}

// The point baseline's pair separation: the same formula without enclosures.
__device__ __forceinline__ pt separated_product(const pt &Z, const pt &W) {
  const pt S = e_add(Z, W), D = e_sub(Z, W);
  const pt A{0.5 * S.re, 0.5 * S.im}, B{0.5 * D.im, -0.5 * D.re};
  return pt{A.re * B.re - A.im * B.im, A.re * B.im + A.im * B.re};
}

// The same in single precision (the naive FP32 baseline).
__device__ __forceinline__ pf separated_product(const pf &Z, const pf &W) {
  const pf S = e_add(Z, W), D = e_sub(Z, W);
  const pf A{0.5f * S.re, 0.5f * S.im}, B{0.5f * D.im, -0.5f * D.re};
  return pf{A.re * B.re - A.im * B.im, A.re * B.im + A.im * B.re};
}

// A product's packed input element a + i b from two digits, thin.
__device__ __forceinline__ void e_thin_pair(ci &z, double da, double db) { z = ci{-da, da, -db, db}; }
__device__ __forceinline__ void e_thin_pair(md &z, double da, double db) { z = md{da, db, 0.0}; }
__device__ __forceinline__ void e_thin_pair(pt &z, double da, double db) { z = pt{da, db}; }
__device__ __forceinline__ void e_thin_pair(pf &z, double da, double db) {
  z = pf{static_cast<float>(da), static_cast<float>(db)};  // digits below 256: exact
}

// Real-part and imaginary-part enclosures (negated lower bound, upper bound).
__device__ __forceinline__ double2 e_re_nh(const ci &z) { return make_double2(z.rn, z.rh); }
__device__ __forceinline__ double2 e_im_nh(const ci &z) { return make_double2(z.in, z.ih); }
__device__ __forceinline__ double2 e_re_nh(const md &z) { return make_double2(md_re_n(z), md_re_h(z)); }
__device__ __forceinline__ double2 e_im_nh(const md &z) { return make_double2(md_im_n(z), md_im_h(z)); }
__device__ __forceinline__ double2 e_re_nh(const pt &z) { return make_double2(-z.re, z.re); }
__device__ __forceinline__ double2 e_im_nh(const pt &z) { return make_double2(-z.im, z.im); }
__device__ __forceinline__ double2 e_re_nh(const pf &z) {
  return make_double2(-static_cast<double>(z.re), static_cast<double>(z.re));
}
__device__ __forceinline__ double2 e_im_nh(const pf &z) {
  return make_double2(-static_cast<double>(z.im), static_cast<double>(z.im));
}

// ---------------------------------------------------------------------------
// k_small: the whole product in one workgroup of N/8 threads, N = 2^log_n,
// 2^9 <= N <= 2^12.  LDS: N half-elements (16 B) for the exchanges, reused for
// the coefficients.

// An FP32 disc as an FP64 element (float to double is exact).
__device__ __forceinline__ void mr_to_e(const mr &a, ci &z) { z = mr_to_ci(a); }
__device__ __forceinline__ void mr_to_e(const mr &a, md &z) {
  z = md{static_cast<double>(a.re), static_cast<double>(a.im), static_cast<double>(a.r)};
}
__device__ __forceinline__ void mr_to_e(const mr &a, pf &z) { z = pf{a.re, a.im}; }  // (unused)
__device__ __forceinline__ void mr_to_e(const mr &a, pt &z) {  // (no FP32 attempt with points)
  z = pt{static_cast<double>(a.re), static_cast<double>(a.im)};
}

// E: rectangles (ci), or discs (md) for the packed transform.
template <int LOG_N, bool WAVE, int PACK, class E>
__device__ __forceinline__ void small_body(const task &tk, int bits, int mode, int fp32, int hooks,
                                           int rerun, const twtab &T, double *dbg, double2 *h,
                                           cert_shared &sh, uint32_t *sh_waves) {
  constexpr int M8 = 1 << (LOG_N - 3);
  constexpr uint32_t mask = (1u << LOG_N) - 1u;
  const int j = threadIdx.x;
  E va[8];
  uint32_t ra[8], rb[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    ra[r] = load_digit(tk.a, tk.nda, j + r * M8, bits);
    rb[r] = load_digit(tk.b, tk.ndb, j + r * M8, bits);
  }
  if constexpr (PACK != 0) {  // one transform of z = a + i b, then separation
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const double da = digit_value(ra[r], tk.nda, j + r * M8, bits);
      const double db = digit_value(rb[r], tk.ndb, j + r * M8, bits);
      e_thin_pair(va[r], da, db);
    }
    if (fp32) {  // forward transform in FP32 discs, then back to FP64 elements
      mr w[8];
#pragma unroll
      for (int r = 0; r < 8; ++r)
        w[r] = mr{static_cast<float>(digit_value(ra[r], tk.nda, j + r * M8, bits)),
                  static_cast<float>(digit_value(rb[r], tk.ndb, j + r * M8, bits)), 0.0f};
      mr_fft8_group<LOG_N, WAVE>(w, j, reinterpret_cast<float4 *>(h), T);
      const float extra = (hooks & HOOK_FORCE_FP32_FAIL) ? 1.0e9f : 0.0f;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        w[r].r += extra;
        mr_to_e(w[r], va[r]);
      }
    } else {
      fft8_group<LOG_N, WAVE, false, twtab, E, false, true>(va, j, h, 0, T);  // thin digits
    }
    // One product per pair {k, -k} (C_{-k} = conj C_k, the coefficients are
    // real): k < N/2 (r < 4) computes it from Z_{-k} and hands it to element
    // -k; k = 0 and k = N/2 (thread 0, r = 0 and 4) are their own partners.
    // Exchanges in 16-byte words through LDS.
    const bool own4 = j == 0;
    uint32_t src[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) src[r] = (0u - static_cast<uint32_t>(j + r * M8)) & mask;
    double2 pr[5];
    xsync<WAVE>();
#pragma unroll
    for (int r = 0; r < 8; ++r)
      if (r >= 4 || own4) h[lpad(j + r * M8)] = e_word0(va[r]);
    xsync<WAVE>();
#pragma unroll
    for (int r = 0; r < 4; ++r) pr[r] = h[lpad(src[r])];
    if (own4) pr[4] = h[lpad(src[4])];
    xsync<WAVE>();
#pragma unroll
    for (int r = 0; r < 8; ++r)
      if (r >= 4 || own4) h[lpad(j + r * M8)] = e_word1(va[r]);
    xsync<WAVE>();
    E C[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      E Zm;  // Z_{-k}
      e_from_words(Zm, pr[r], h[lpad(src[r])]);
      C[r] = separated_product(va[r], e_conj(Zm));
    }
    if (own4) {
      E Zm;
      e_from_words(Zm, pr[4], h[lpad(src[4])]);
      va[4] = e_conj(separated_product(va[4], e_conj(Zm)));
    }
    double2 t0[4];
    xsync<WAVE>();
#pragma unroll
    for (int r = 0; r < 4; ++r) h[lpad(src[r])] = e_word0(C[r]);
    xsync<WAVE>();
#pragma unroll
    for (int r = 4; r < 8; ++r) t0[r - 4] = h[lpad(j + r * M8)];
    xsync<WAVE>();
#pragma unroll
    for (int r = 0; r < 4; ++r) h[lpad(src[r])] = e_word1(C[r]);
    xsync<WAVE>();
#pragma unroll
    for (int r = 4; r < 8; ++r)
      if (r != 4 || !own4) e_from_words(va[r], t0[r - 4], h[lpad(j + r * M8)]);
#pragma unroll
    for (int r = 0; r < 4; ++r) va[r] = e_conj(C[r]);
  } else {  // one transform per operand, pointwise product
    ci vb[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      va[r] = ci_thin_real(digit_value(ra[r], tk.nda, j + r * M8, bits));
      vb[r] = ci_thin_real(digit_value(rb[r], tk.ndb, j + r * M8, bits));
    }
    if (fp32) {
      const float extra = (hooks & HOOK_FORCE_FP32_FAIL) ? 1.0e9f : 0.0f;
      mr w[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) w[r] = mr{static_cast<float>(va[r].rh), 0.0f, 0.0f};
      mr_fft8_group<LOG_N, WAVE>(w, j, reinterpret_cast<float4 *>(h), T);
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        w[r].r += extra;
        va[r] = mr_to_ci(w[r]);
      }
#pragma unroll
      for (int r = 0; r < 8; ++r) w[r] = mr{static_cast<float>(vb[r].rh), 0.0f, 0.0f};
      mr_fft8_group<LOG_N, WAVE>(w, j, reinterpret_cast<float4 *>(h), T);
#pragma unroll
      for (int r = 0; r < 8; ++r) vb[r] = mr_to_ci(w[r]);
    } else {
      fft8_group<LOG_N, WAVE, false, twtab, ci, false, true>(va, j, h, 0, T);  // thin digits
      fft8_group<LOG_N, WAVE, false, twtab, ci, false, true>(vb, j, h, 0, T);
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) va[r] = ci_conj(ci_mul_fast(va[r], vb[r]));
  }
  fft8_group<LOG_N, WAVE>(va, j, h, 0, T);
  const double scale = ldexp(1.0, -LOG_N);
  cert_acc acc{0.0, 0u, 0u, 0u};
  unsigned long long cv[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const uint32_t i = j + r * M8;
    const E v = e_scale(e_conj(va[r]), scale);
    const double2 re = e_re_nh(v), im = e_im_nh(v);
    if (dbg != nullptr && blockIdx.x == 0) dbg_store(dbg, i, ci{re.x, re.y, im.x, im.y});
    if constexpr (e_traits<E>::rigorous) {
      // a real coefficient: the imaginary part must contain 0
      cv[r] = certify_re(re.x, re.y, im.x >= 0.0 && im.y >= 0.0, i, tk.L, mode, acc);
    } else {
      cv[r] = naive_round(re.y, i, tk.L, acc);
    }
  }
  cert_reduce(sh, acc);
  __syncthreads();  // LDS free again; counters final
  unsigned long long *cl = reinterpret_cast<unsigned long long *>(h);
#pragma unroll
  for (int r = 0; r < 8; ++r) cl[j + r * M8] = cv[r];
  __syncthreads();
  const bool failed = (sh.too_wide + sh.internal) != 0u;
  const uint32_t L = tk.L;
  const uint32_t nout = tk.na + tk.nb;
  // waves = N/512, 9 chunks of 64 per wave cover 9N/8 >= N + 1 >= nout positions
  if (bits == 8) {
    auto C = [&](long long q) -> unsigned long long {
      return (q >= 0 && q < static_cast<long long>(L)) ? cl[q] : 0ull;
    };
    carry_block<9>(C, 0, nout, tk.out, failed, [](uint32_t, uint32_t) { return 0u; }, sh_waves);
  } else {
    auto C = [&](long long q) -> unsigned long long {
      if (q < 0) return 0ull;
      const long long i0 = 2 * q, i1 = 2 * q + 1;
      const unsigned long long lo = i0 < static_cast<long long>(L) ? cl[i0] : 0ull;
      const unsigned long long hi = i1 < static_cast<long long>(L) ? cl[i1] : 0ull;
      return lo + 16ull * hi;
    };
    carry_block<9>(C, 0, nout, tk.out, failed, [](uint32_t, uint32_t) { return 0u; }, sh_waves);
  }
  if (threadIdx.x == 0) {
    dev_stats *st = tk.st;
    st->max_rad_bits = sh.rad_bits;
    st->half_int = sh.half;
    st->too_wide = sh.too_wide;
    st->internal = sh.internal;
    st->carry_err = 0u;
    st->fallback = (rerun && tk.fp32 != 0u) ? 1u : 0u;
    st->fp32 = tk.fp32;
  }
}

// One product per workgroup.  fp32: first attempt with FP32 forward
// transforms (every task of the launch is marked for it); rerun: the FP64
// launch that follows such an attempt over the whole length class, where the
// marked products that the attempt certified return at once.  The decision is
// read from the statistics on the device, so a captured launch sequence holds
// the fallback unconditionally.
// The packed kernel's registers are capped at 128 (four waves per SIMD; a few
// values spill).  At 2^12 points a workgroup is 8 waves with 72 KB of LDS, and
// two fit a CU only at four waves per SIMD: 36% more products per second than
// at the uncapped 137 registers; 5-7% more at 2^9..2^11.
template <int LOG_N, int bits, int pack, class E>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(pack == 1 ? 4 : 1)))
void k_small(const task *tasks, int mode, int fp32, int rerun, int hooks, twtab T, double *dbg) {
  extern __shared__ double2 hbuf[];
  __shared__ cert_shared sh;
  __shared__ uint32_t sh_waves[8];
  const uint32_t z = enter_mode<E>();
  const task tk = after_mode(tasks, z)[blockIdx.x];
  T.tab = after_mode(T.tab, z);
  if (rerun && tk.fp32 != 0u && tk.st->too_wide == 0u && tk.st->internal == 0u) return;
  if (threadIdx.x == 0) sh = cert_shared{0ull, 0ull, 0u, 0u};
  __syncthreads();
  small_body<LOG_N, (LOG_N <= 9), pack, E>(tk, bits, mode, fp32, hooks, rerun, T, dbg, hbuf, sh,
                                           sh_waves);
}

// ---------------------------------------------------------------------------
// Multi-pass kernels.
//
// Pass order over the products of a launch alternates: the column passes and
// the single-workgroup products take products in ascending order, the row pass
// and the carry scan in descending order.  Each pass therefore starts on the
// products whose data the previous pass wrote last, which are still held in
// the last-level cache (256 MB Infinity Cache on MI355X) when a launch's
// arrays are larger than it.

// Inter-pass twiddle omega_N^t, t = (a * b) mod N, as the product of two table
// entries: the two factors come from 2^(log_n - h) and 2^h contiguous entries,
// which stay cache-resident, instead of one scattered read over all N entries.
// The product's error has one bound for every pair (pass_tw_bound).
// UH: the caller guarantees t < N/2.  Then the root lies in the upper half
// plane and so does the computed point: its sine is either exactly 0 (t = 0)
// or at least sin(2 pi/N) > 10^-6 for N <= 2^22, far above the product's
// rounding, so the known-sign form of the rotation applies.
template <bool UH = false, class E>
__device__ __forceinline__ E apply_pass_tw(const E &v, const twtab &T, uint32_t a, uint32_t b,
                                           int log_n) {
  const uint32_t t = (a * b) & ((1u << log_n) - 1u);
  const int h = (log_n + 1) >> 1;
  // omega_N^t = omega_{N / 2^h}^{t >> h} * omega_N^{t mod 2^h}
  const double2 w = tw_point_product(root(T, log_n - h, t >> h), root(T, log_n, t & ((1u << h) - 1u)));
  return UH ? e_tw_uh(v, w.x, w.y, pass_tw_bound(T.e)) : e_tw(v, w.x, w.y, pass_tw_bound(T.e));
}


// Keeps the compiler from interleaving the final stores with the twiddle loads
// before them: one counter tracks both loads and stores, so a load issued
// after a store cannot be waited for without also waiting for that store, and
// each interleaved pair would cost a full memory round trip.
__device__ __forceinline__ void stores_after_loads() { __builtin_amdgcn_sched_barrier(0); }

// ---------------------------------------------------------------------------
// Intermediate arrays between the passes of a product: 20 bytes per element
// instead of 32.  Element idx of a transform array of N elements is kept as its
// midpoint (m_re, m_im), a double2 at m[idx], and one radius r at least both
// half-widths, as the high word of r's binary64 pattern rounded up (for r >= 0
// the patterns order like the values), a uint32 at r[idx]; the radii follow the
// N midpoints in the same buffer.  Read back as [m - r, m + r] rounded outward,
// the element encloses the interval that was stored; the price is the
// midpoint's rounding and one radius for both parts.
struct mrbuf {
  d2v *m;
  uint32_t *r;
};
__device__ __forceinline__ mrbuf mr_of(ci *y, int log_n) {
  return mrbuf{reinterpret_cast<d2v *>(y), reinterpret_cast<uint32_t *>(y + (size_t(1) << (log_n - 1)))};
}
struct mr_raw {
  d2v m;
  uint32_t r;
};
__device__ __forceinline__ mr_raw mr_load_raw(const mrbuf &b, size_t idx) {
  return mr_raw{gload(b.m + idx), gload(b.r + idx)};
}
// A disc is stored as it is (only its radius rounded up to 32 bits).
__device__ __forceinline__ double mr_radius(uint32_t w) {
  return __longlong_as_double(static_cast<long long>(static_cast<unsigned long long>(w) << 32));
}
__device__ __forceinline__ void mr_decode(const mr_raw &x, ci &z) {
  const double r = mr_radius(x.r);
  z = ci{ru_sub(r, x.m.x), ru_add(x.m.x, r), ru_sub(r, x.m.y), ru_add(x.m.y, r)};
}
__device__ __forceinline__ void mr_decode(const mr_raw &x, md &z) { z = md{x.m.x, x.m.y, mr_radius(x.r)}; }
template <class E> __device__ __forceinline__ E mr_load(const mrbuf &b, size_t idx) {
  E z;
  mr_decode(mr_load_raw(b, idx), z);
  return z;
}
__device__ __forceinline__ void mr_put(const mrbuf &b, size_t idx, double mre, double mim, double r) {
  const unsigned long long bits = static_cast<unsigned long long>(__double_as_longlong(r)) + 0xFFFFFFFFull;
  gstore(b.m + idx, d2v{mre, mim});
  gstore(b.r + idx, static_cast<uint32_t>(bits >> 32));
}
__device__ __forceinline__ void mr_store(const mrbuf &b, size_t idx, const ci &v) {
  const double mre = ru_mul(0.5, ru_sub(v.rh, v.rn)), mim = ru_mul(0.5, ru_sub(v.ih, v.in));
  const double r = dmax(dmax(ru_sub(v.rh, mre), ru_add(v.rn, mre)), dmax(ru_sub(v.ih, mim), ru_add(v.in, mim)));
  mr_put(b, idx, mre, mim, r);
}
__device__ __forceinline__ void mr_store(const mrbuf &b, size_t idx, const md &v) {
  mr_put(b, idx, v.re, v.im, v.r);
}
// The point baseline keeps the midpoints only.
template <> __device__ __forceinline__ pt mr_load<pt>(const mrbuf &b, size_t idx) {
  const d2v m = gload(b.m + idx);
  return pt{m.x, m.y};
}
__device__ __forceinline__ void mr_store(const mrbuf &b, size_t idx, const pt &v) {
  gstore(b.m + idx, d2v{v.re, v.im});
}

// Half-length inverse of a spectrum Z whose inverse transform x is real (the
// product's coefficients): y_m = x_{2m} + i x_{2m+1}, m < N/2, is the
// length-N/2 inverse DFT of
//   U_k = (Z_k + Z_{k+N/2}) + i omega_N^{-k} (Z_k - Z_{k+N/2}),   k < N/2,
// scaled by 1/N (split the inverse sum over even and odd n).  The inverse runs
// as the forward DFT of the conjugate, so the rows work on P = conj Z_k and
// Q = conj Z_{k+N/2}:  conj U_k = (P + Q) - i omega_N^k (P - Q).  An enclosure
// of y is one of x: its real part encloses x_{2m} and its imaginary part
// x_{2m+1}, because the exact x is real.  w is omega_N^k as a point within
// ew of the root; k < N/2 puts it in the upper half plane (see apply_pass_tw).
template <class E>
__device__ __forceinline__ E half_inverse_input(const E &P, const E &Q, double2 w, double ew) {
  const E t = e_tw_uh(e_sub(P, Q), w.x, w.y, ew);
  return e_add(e_add(P, Q), e_mul_negi(t));
}

// Row k1 of the half-length inverse: v[r] holds P at k2 = j + r N2/8 (r < 8),
// so that Z_{k+N/2} (k2 + N2/2, same row) sits in the same thread (r + 4).
// Forms conj U for k2 < N2/2, runs the length-N2/2 row DFT and the conjugate
// inter-pass twiddle of the length-N/2 four-step inverse, omega_{N/2}^{n2 k1},
// and stores the N2/2 results at the start of the row.  `h` is the row's
// exchange buffer (N2/2 elements), TF the table the row DFT reads.
template <int LOG_N2, bool WAVE, class TT, class E>
__device__ __forceinline__ void half_inverse_row(const E v[8], int j, uint32_t k1, int log_n1,
                                                 double2 *h, const TT &TF, const twtab &T,
                                                 const mrbuf &Y) {
  constexpr int M8 = 1 << (LOG_N2 - 3);
  const int log_n = log_n1 + LOG_N2;
  // omega_N^k for k = k1 + N1 k2 is omega_N^{k1} omega_{N2}^{k2}, two table
  // entries (the bound pass_tw_bound covers their product); the first is the
  // same for the whole row (one address for the wavefront when the row is
  // whole wavefronts)
  const uint32_t k1u = M8 >= 64 ? __builtin_amdgcn_readfirstlane(k1) : k1;
  const double2 w1 = root(T, log_n, k1u);
  E u[4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
    u[r] = half_inverse_input(v[r], v[r + 4],
                              tw_point_product(w1, root(T, LOG_N2, static_cast<uint32_t>(j + r * M8))),
                              pass_tw_bound(T.e));
  fft4_group<LOG_N2 - 1, WAVE>(u, j, h, TF);
#pragma unroll
  for (int q = 0; q < 4; ++q)  // n2 k1 < N/4 for q < 2: the upper half plane
    u[q] = e_conj(q < 2 ? apply_pass_tw<true>(u[q], T, j + q * M8, k1, log_n - 1)
                        : apply_pass_tw(u[q], T, j + q * M8, k1, log_n - 1));
  stores_after_loads();
  const size_t row = static_cast<size_t>(k1) << LOG_N2;
#pragma unroll
  for (int q = 0; q < 4; ++q) mr_store(Y, row + j + q * M8, u[q]);
}

// Column group of a column-pass workgroup, XCD-aware.  Workgroups go round-robin
// over the 8 XCDs (linear id mod 8; with G a multiple of 8, blockIdx.x mod 8),
// so block x takes group (x mod 8) (G/8) + x/8: the groups one XCD runs are
// adjacent in memory, and the cache lines that two neighbouring groups share
// meet in that XCD's L2 instead of travelling to two of them.
__device__ __forceinline__ uint32_t xcd_group(uint32_t x, uint32_t G) {
  return (G & 7u) ? x : (x & 7u) * (G >> 3) + (x >> 3);
}

// Statistics and carry-scan state of a product are reset by its first pass.
__device__ __forceinline__ void reset_product_state(const task &tk) {
  if (threadIdx.x == 0) {
    tk.st->max_rad_bits = 0ull;
    tk.st->half_int = 0ull;
    tk.st->too_wide = 0u;
    tk.st->internal = 0u;
    tk.st->carry_err = 0u;
    tk.st->fallback = 0u;
    tk.st->fp32 = 0u;
  }
  for (uint32_t t = threadIdx.x; t < tk.ntiles; t += blockDim.x) tk.tiles[t * TILE_WORD_STRIDE] = 0u;
}

// Columns: thread (c, j) with c = tid % C fastest, so that the C = 2^lc columns
// of a workgroup are adjacent in memory.  grid = (N2 / C, 1 (packed) or 2, tasks).
// The packing and the digit size are compile-time (14% fewer instructions than
// run-time flags: the digit loads then need no branches).
// E: the element type, rectangles (ci) or discs (md, packed transforms only).
template <int LOG_N1, int pack, int bits, class E>
__global__ __launch_bounds__(512) void k_col_fwd(const task *tasks, int log_n2, int lc, twtab T) {
  extern __shared__ double2 hbuf[];
  const uint32_t z = enter_mode<E>();
  const task tk = after_mode(tasks, z)[blockIdx.z];
  T.tab = after_mode(T.tab, z);
  const int log_n = LOG_N1 + log_n2;
  constexpr int M8 = 1 << (LOG_N1 - 3);
  const int c = threadIdx.x & ((1 << lc) - 1), j = threadIdx.x >> lc;
  const uint32_t n2 = (xcd_group(blockIdx.x, gridDim.x) << lc) + c;
  const bool opb = blockIdx.y != 0;
  if (blockIdx.x == 0 && !opb) reset_product_state(tk);
  uint32_t idx[8], ra[8], rb[8];
  const uint8_t *p = opb ? tk.b : tk.a;
  const uint32_t nd = opb ? tk.ndb : tk.nda;
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    idx[r] = (static_cast<uint32_t>(j + r * M8) << log_n2) + n2;
    ra[r] = load_digit(pack ? tk.a : p, pack ? tk.nda : nd, idx[r], bits);
    if (pack) rb[r] = load_digit(tk.b, tk.ndb, idx[r], bits);
  }
  E v[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    if constexpr (pack != 0) {  // z = a + i b: both real operands in one complex transform
      const double da = digit_value(ra[r], tk.nda, idx[r], bits);
      const double db = digit_value(rb[r], tk.ndb, idx[r], bits);
      e_thin_pair(v[r], da, db);
    } else {
      v[r] = ci_thin_real(digit_value(ra[r], nd, idx[r], bits));
    }
  }
  fft8_group<LOG_N1, false, false, twtab, E, false, true>(v, j, hbuf + c, lc, T);  // thin digits
  const mrbuf Y = mr_of(opb ? tk.yb : tk.ya, log_n);
#pragma unroll
  for (int q = 0; q < 8; ++q) v[q] = apply_pass_tw(v[q], T, n2, j + q * M8, log_n);
  stores_after_loads();
#pragma unroll
  for (int q = 0; q < 8; ++q) mr_store(Y, (static_cast<size_t>(j + q * M8) << log_n2) + n2, v[q]);
}

// Rows (one transform per operand): R rows k1 per workgroup, N2/8 threads per
// row.  grid = (N1 / R, tasks).
template <int LOG_N2, bool WAVE>
__device__ __forceinline__ void row_body(const task &tk, int log_n1, int R, const twtab &T,
                                         double2 *hbuf) {
  const int log_n = log_n1 + LOG_N2;
  constexpr int M8 = 1 << (LOG_N2 - 3);
  const int g = threadIdx.x / M8, j = threadIdx.x % M8;
  const uint32_t k1 = blockIdx.x * R + g;
  double2 *hg = hbuf + static_cast<size_t>(g) * lpad_size(size_t(1) << LOG_N2);
  const size_t row = static_cast<size_t>(k1) << LOG_N2;
  ci va[8], vb[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    va[r] = mr_load<ci>(mr_of(tk.ya, log_n), row + j + r * M8);
    vb[r] = mr_load<ci>(mr_of(tk.yb, log_n), row + j + r * M8);
  }
  fft8_group<LOG_N2, WAVE>(va, j, hg, 0, T);
  fft8_group<LOG_N2, WAVE>(vb, j, hg, 0, T);
#pragma unroll
  for (int r = 0; r < 8; ++r) va[r] = ci_conj(ci_mul_fast(va[r], vb[r]));
  half_inverse_row<LOG_N2, WAVE>(va, j, k1, log_n1, hg, T, T, mr_of(tk.ya, log_n));
}

template <int LOG_N2>
__global__ __launch_bounds__(512) void k_row(const task *tasks, int log_n1, int R, twtab T) {
  extern __shared__ double2 hbuf[];
  const uint32_t z = enter_round_up();
  const task tk = after_mode(tasks, z)[gridDim.y - 1 - blockIdx.y];  // last written first
  T.tab = after_mode(T.tab, z);
  row_body<LOG_N2, (LOG_N2 <= 9)>(tk, log_n1, R, T, hbuf);
}

// Row pairs for the packed transform.  Index k = k1 + N1 k2 has
// -k = (N1 - k1) + N1 (N2 - 1 - k2) for k1 > 0 and -k = N1 ((N2 - k2) mod N2) for
// k1 = 0, so the partner Z_{-k} of every element of rows k1 and N1 - k1 lies in
// the other row (pair p >= 1, rows p and N1 - p), and rows 0 and N1/2 are their
// own partners (pair 0).  A workgroup holds G pairs, each as two row groups of
// N2/8 threads.  Per row: forward length-N2 DFT, separated pointwise product
// with the partner row, then the row step of the half-length inverse
// (half_inverse_row).  grid = (N1 / 2 / G, tasks).
template <int LOG_N2, bool WAVE, class E>
__device__ __forceinline__ void row_pair_body(const task &tk, int log_n1, int G, const twtab &T,
                                              double2 *hbuf) {
  const int log_n = log_n1 + LOG_N2;
  constexpr uint32_t N2 = 1u << LOG_N2;
  const uint32_t N1 = 1u << log_n1;
  constexpr int M8 = 1 << (LOG_N2 - 3);
  const int rg = threadIdx.x / M8;  // row group in the workgroup
  const int j = threadIdx.x % M8;
  const int g = rg >> 1, role = rg & 1;
  const uint32_t p = blockIdx.x * G + g;
  const bool self = p == 0;
  const uint32_t k1 = role == 0 ? p : (self ? N1 / 2 : N1 - p);
  constexpr size_t rowslots = lpad_size(size_t(1) << LOG_N2);
  // rows of at most 2^8 points: the pair's two row groups (2 N2/8 <= 64
  // threads) are one wavefront, whose LDS operations complete in order, so
  // the partner exchange needs no workgroup barrier
  constexpr bool PW = LOG_N2 <= 8;
  double2 *hown = hbuf + static_cast<size_t>(rg) * rowslots;
  double2 *hpart = self ? hown : hbuf + static_cast<size_t>(rg ^ 1) * rowslots;
  const size_t row = static_cast<size_t>(k1) << LOG_N2;
  E v[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) v[r] = mr_load<E>(mr_of(tk.ya, log_n), row + j + r * M8);
  fft8_group<LOG_N2, WAVE, true>(v, j, hown, 0, T);  // stage twiddles loaded a stage ahead
  // Each pair {k, -k} of the two rows needs one product: C_{-k} = conj(C_k)
  // (the coefficients are real).  Elements k2 < N2/2 (r < 4) compute it from
  // their partner's value, and hand it to the partner, whose element lies in
  // the other half (k2 >= N2/2) -- except in row 0, where k2 = 0 and k2 = N2/2
  // are their own partners (both held by thread 0).  The exchange goes through
  // the row buffers, free once the row DFT is done: each row's elements
  // k2 >= N2/2 sit at slot w N2/2 + (k2 - N2/2) for their two 16-byte words w
  // (k2 = 0 of row 0 at the spare slots N2, N2 + 1).  Every slot is read by one
  // thread only (the partner of its element), and that thread writes the
  // product back into the very slot it read, so the exchange needs just two
  // barriers when the partner row is another wavefront: after the values are
  // written, and after the products are.
  constexpr uint32_t H2 = N2 / 2;
  constexpr bool TWO = e_traits<E>::words == 2;
  const bool own4 = k1 == 0 && j == 0;
  int ps[4];  // slot of Z_{-k} for r < 4 (in the partner's buffer)
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const uint32_t k2 = j + r * M8;
    const uint32_t m = k1 == 0 ? ((N2 - k2) & (N2 - 1)) : (N2 - 1 - k2);  // -k's column
    ps[r] = r == 0 && own4 ? static_cast<int>(N2) : static_cast<int>(m - H2);
  }
  // k2 = N2/2 of row 0 is its own partner: its final value, computed here,
  // goes out and comes back unchanged (no thread reads its slot as a partner)
  if (own4) v[4] = e_conj(separated_product(v[4], e_conj(v[4])));
  if constexpr (!WAVE) xsync<false>();  // the row's other waves are done with the DFT's exchanges
#pragma unroll
  for (int r = 4; r < 8; ++r) {
    const int e = j + (r - 4) * M8;
    hown[e] = e_word0(v[r]);
    if constexpr (TWO) hown[H2 + e] = e_word1(v[r]);
  }
  if (own4) {
    hown[N2] = e_word0(v[0]);
    if constexpr (TWO) hown[N2 + 1] = e_word1(v[0]);
  }
  xsync<PW>();
  E C[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int w1 = ps[r] == static_cast<int>(N2) ? static_cast<int>(N2 + 1) : static_cast<int>(H2) + ps[r];
    E Zm;  // Z_{-k}
    e_from_words(Zm, hpart[ps[r]], TWO ? hpart[w1] : make_double2(0.0, 0.0));
    C[r] = separated_product(v[r], e_conj(Zm));
    // element -k receives conj(C_{-k}) = C_k, in the slot its value came from
    hpart[ps[r]] = e_word0(C[r]);
    if constexpr (TWO) hpart[w1] = e_word1(C[r]);
  }
  xsync<PW>();
#pragma unroll
  for (int r = 4; r < 8; ++r) {
    const int e = j + (r - 4) * M8;
    e_from_words(v[r], hown[e], TWO ? hown[H2 + e] : make_double2(0.0, 0.0));
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) v[r] = e_conj(C[r]);
  // (the row DFT of the inverse synchronises before its first write to hown)
  half_inverse_row<LOG_N2, WAVE>(v, j, k1, log_n1, hown, T, T, mr_of(tk.ya, log_n));
}

template <int LOG_N2, class E>
// Rows of up to 2^9 points: four waves per SIMD (registers capped at 128, no
// spills), the stage twiddles of both row DFTs loaded a stage ahead.  Longer
// rows: three waves (168 registers), which measured faster than two.
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(LOG_N2 <= 9 ? 4 : 3))) void k_row_pair(const task *tasks, int log_n1, int G, twtab T) {
  extern __shared__ double2 hbuf[];
  const uint32_t z = enter_mode<E>();
  const task tk = after_mode(tasks, z)[gridDim.y - 1 - blockIdx.y];  // last written first
  T.tab = after_mode(T.tab, z);
  row_pair_body<LOG_N2, (LOG_N2 <= 9), E>(tk, log_n1, G, T, hbuf);
}

// Persistent form of k_row_pair for rows of at most 2^9 points: gridDim.x
// workgroups (as many as are resident at once) walk the (product, pair group)
// items, products in descending order, and each prefetches the next item's rows
// into registers while it computes the current one, so that the global-memory
// latency of one item overlaps the arithmetic of the previous one.  The
// twiddles of the row DFTs are copied once into LDS (levels up to 2^LOG_N2), so
// the stage twiddle reads do not wait behind the stores of the previous item
// (one counter tracks both global loads and stores).
template <int LOG_N2>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2))) void k_row_pair_p(
    const task *tasks, int ntasks, int log_n1, int G, twtab T) {
  static_assert(LOG_N2 <= 9, "rows of one wavefront");
  extern __shared__ double2 hbuf[];
  const uint32_t z = enter_round_up();
  tasks = after_mode(tasks, z);
  T.tab = after_mode(T.tab, z);
  constexpr uint32_t N2 = 1u << LOG_N2;
  constexpr int M8 = 1 << (LOG_N2 - 3);
  constexpr size_t rowslots = lpad_size(size_t(1) << LOG_N2);
  const int log_n = log_n1 + LOG_N2;
  const uint32_t N1 = 1u << log_n1;
  const int rg = threadIdx.x / M8, j = threadIdx.x % M8;
  const int g = rg >> 1, role = rg & 1;
  const uint32_t per_task = N1 / 2 / G, total = per_task * ntasks;
  double2 *tl = hbuf + static_cast<size_t>(2 * G) * rowslots;
  for (uint32_t i = threadIdx.x; i < (2u << LOG_N2); i += blockDim.x) tl[i] = T.tab[i];
  __syncthreads();
  const twtab_lds TL{(lds_dp)(reinterpret_cast<double *>(tl)), LOG_N2, T.e};
  uint32_t it = blockIdx.x;
  if (it >= total) return;  // uniform over the workgroup
  // item -> (product, row k1 of this thread's row group)
  const auto locate = [&](uint32_t item, const task *&tk, uint32_t &k1, bool &self) {
    tk = tasks + (ntasks - 1 - item / per_task);
    const uint32_t p = (item % per_task) * G + g;
    self = p == 0;
    k1 = role == 0 ? p : (self ? N1 / 2 : N1 - p);
  };
  const task *tk;
  uint32_t k1;
  bool self;
  locate(it, tk, k1, self);
  ci v[8];
  mr_raw nx[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) v[r] = mr_load<ci>(mr_of(tk->ya, log_n), (static_cast<size_t>(k1) << LOG_N2) + j + r * M8);
  for (;;) {
    const uint32_t nit = it + gridDim.x;
    const bool more = nit < total;
    const task *ntk = tk;
    uint32_t nk1 = k1;
    bool nself = self;
    if (more) {
      locate(nit, ntk, nk1, nself);
#pragma unroll
      for (int r = 0; r < 8; ++r)
        nx[r] = mr_load_raw(mr_of(ntk->ya, log_n), (static_cast<size_t>(nk1) << LOG_N2) + j + r * M8);
    }
    double2 *hown = hbuf + static_cast<size_t>(rg) * rowslots;
    double2 *hpart = self ? hown : hbuf + static_cast<size_t>(rg ^ 1) * rowslots;
    fft8_group<LOG_N2, true>(v, j, hown, 0, TL);
    uint32_t src[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const uint32_t k2 = j + r * M8;
      src[r] = k1 == 0 ? ((N2 - k2) & (N2 - 1)) : (N2 - 1 - k2);
    }
    double2 pr[8];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 8; ++r) hown[lpad(j + r * M8)] = make_double2(v[r].rn, v[r].rh);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 8; ++r) pr[r] = hpart[lpad(src[r])];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 8; ++r) hown[lpad(j + r * M8)] = make_double2(v[r].in, v[r].ih);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const double2 pi = hpart[lpad(src[r])];
      const ci W{pr[r].x, pr[r].y, pi.y, pi.x};  // conj(Z_{-k})
      v[r] = ci_conj(separated_product(v[r], W));
    }
    __syncthreads();  // the partner has read this row's buffer
    half_inverse_row<LOG_N2, true>(v, j, k1, log_n1, hown, TL, T, mr_of(tk->ya, log_n));
    if (!more) break;
    it = nit;
    tk = ntk;
    k1 = nk1;
    self = nself;
#pragma unroll
    for (int r = 0; r < 8; ++r) mr_decode(nx[r], v[r]);
  }
}

// Inverse columns of the half-length inverse + scale + certification.  The
// rows left y's four-step intermediate in the first N2/2 entries of every row;
// column n2 < N2/2 gives y_{n2 + (N2/2) n1} = x_{2 m} + i x_{2 m + 1} with
// 2 m = N2 n1 + 2 n2, and each part is certified as one coefficient.
// grid = (N2 / 2 / C, tasks).
// Rectangles, columns of 2^7 points and more: each stage twiddle loaded right
// where it is used, which keeps the kernel at 124-126 registers (four waves
// per SIMD, no spills): 6.5% faster than three waves at 136 registers with a
// stage's twiddles loaded together (64 products at 2^18).  Discs measured
// slower that way and keep the default; at 2^6 the cap would spill.
template <int LOG_N1, class E>
__global__ __launch_bounds__(512)
__attribute__((amdgpu_waves_per_eu(std::is_same<E, ci>::value && LOG_N1 >= 7 ? 4 : 2)))
void k_col_inv(const task *tasks, int log_n2, int lc, int mode,
                                                 twtab T, double *dbg) {
  extern __shared__ double2 hbuf[];
  __shared__ cert_shared sh;
  const uint32_t z = enter_mode<E>();
  const task tk = after_mode(tasks, z)[blockIdx.y];
  T.tab = after_mode(T.tab, z);
  const int log_n = LOG_N1 + log_n2;
  constexpr int M8 = 1 << (LOG_N1 - 3);
  const int c = threadIdx.x & ((1 << lc) - 1), j = threadIdx.x >> lc;
  const uint32_t n2 = (xcd_group(blockIdx.x, gridDim.x) << lc) + c;
  if (threadIdx.x == 0) sh = cert_shared{0ull, 0ull, 0u, 0u};
  E v[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const uint32_t k1 = j + r * M8;
    v[r] = e_conj(mr_load<E>(mr_of(tk.ya, log_n), (static_cast<size_t>(k1) << log_n2) + n2));
  }
  fft8_group<LOG_N1, false, false, twtab, E, std::is_same<E, ci>::value>(v, j, hbuf + c, lc, T);
  const double scale = ldexp(1.0, -log_n);
  cert_acc acc{0.0, 0u, 0u, 0u};
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const uint32_t n1 = j + q * M8;
    const uint32_t i = (n1 << log_n2) + 2 * n2;
    const E w = e_scale(e_conj(v[q]), scale);
    const double2 re = e_re_nh(w), im = e_im_nh(w);
    if (dbg != nullptr && blockIdx.y == 0) {
      dbg_store(dbg, i, ci{re.x, re.y, 0.0, 0.0});
      dbg_store(dbg, i + 1, ci{im.x, im.y, 0.0, 0.0});
    }
    unsigned long long c0, c1;
    if constexpr (e_traits<E>::rigorous) {
      c0 = certify_re(re.x, re.y, true, i, tk.L, mode, acc);
      c1 = certify_re(im.x, im.y, true, i + 1, tk.L, mode, acc);
    } else {
      c0 = naive_round(re.y, i, tk.L, acc);
      c1 = naive_round(im.y, i + 1, tk.L, acc);
    }
    if (i + 1 < tk.L) {
      u64x2 pair;
      pair.x = c0;
      pair.y = c1;
      gstore(reinterpret_cast<u64x2 *>(tk.c + i), pair);
    } else if (i < tk.L) {
      gstore(tk.c + i, c0);
    }
  }
  cert_reduce(sh, acc);
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicMax(&tk.st->max_rad_bits, sh.rad_bits);
    if (sh.half) atomicAdd(&tk.st->half_int, sh.half);
    if (sh.too_wide) atomicAdd(&tk.st->too_wide, sh.too_wide);
    if (sh.internal) atomicAdd(&tk.st->internal, sh.internal);
  }
}

// ---------------------------------------------------------------------------
// Batched forward interval DFT (section 2.2) of caller-supplied intervals, the
// same two passes as the product's forward transform without the digits.
// Public element layout: 4 doubles {re_lo, re_hi, im_lo, im_hi}; lower bounds
// are negated on load and back on store (exact).

__device__ __forceinline__ ci load_public(const double *x, size_t idx) {
  const ci v = gld(reinterpret_cast<const ci *>(x), idx);  // {re_lo, re_hi, im_lo, im_hi}
  return ci{-v.rn, v.rh, -v.in, v.ih};
}
__device__ __forceinline__ void store_public(double *y, size_t idx, const ci &v) {
  gst(reinterpret_cast<ci *>(y), idx, ci{-v.rn, v.rh, -v.in, v.ih});
}

// Columns: length-N1 DFTs over n1 of x[n1 N2 + n2], times omega_N^{n2 k1}, to
// y[k1 N2 + n2].  Thread (c, j), C = 2^lc adjacent columns per workgroup.
// grid = (N2 / C, vectors).
template <int LOG_N1>
__global__ __launch_bounds__(512) void k_fft_col(const double *x, double *y, int log_n2, int lc,
                                                 twtab T) {
  extern __shared__ double2 hbuf[];
  const uint32_t z = enter_round_up();
  x = after_mode(x, z);
  T.tab = after_mode(T.tab, z);
  const int log_n = LOG_N1 + log_n2;
  constexpr int M8 = 1 << (LOG_N1 - 3);
  const int c = threadIdx.x & ((1 << lc) - 1), j = threadIdx.x >> lc;
  const uint32_t n2 = (xcd_group(blockIdx.x, gridDim.x) << lc) + c;
  const size_t base = static_cast<size_t>(blockIdx.y) << log_n;
  ci v[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) v[r] = load_public(x, base + (static_cast<size_t>(j + r * M8) << log_n2) + n2);
  fft8_group<LOG_N1, false>(v, j, hbuf + c, lc, T);
#pragma unroll
  for (int q = 0; q < 8; ++q)  // n2 k1 < N/2 for q < 4: the upper half plane
    v[q] = q < 4 ? apply_pass_tw<true>(v[q], T, n2, j + q * M8, log_n)
                 : apply_pass_tw(v[q], T, n2, j + q * M8, log_n);
  stores_after_loads();
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const ci w = v[q];
    gst(reinterpret_cast<ci *>(y), base + (static_cast<size_t>(j + q * M8) << log_n2) + n2, w);
  }
}

// Rows, in place: length-N2 DFT of row k1, element k2 of the row then encloses
// X[k1 + N1 k2].  R rows per workgroup, N2/8 threads per row.  grid = (N1 / R,
// vectors).
template <int LOG_N2>
__global__ __launch_bounds__(512) void k_fft_row(double *y, int log_n1, int R, twtab T) {
  extern __shared__ double2 hbuf[];
  const uint32_t z = enter_round_up();
  y = after_mode(y, z);
  T.tab = after_mode(T.tab, z);
  constexpr int M8 = 1 << (LOG_N2 - 3);
  const int g = threadIdx.x / M8, j = threadIdx.x % M8;
  const uint32_t k1 = blockIdx.x * R + g;
  double2 *hg = hbuf + static_cast<size_t>(g) * lpad_size(size_t(1) << LOG_N2);
  const size_t row = (static_cast<size_t>(blockIdx.y) << (log_n1 + LOG_N2)) +
                     (static_cast<size_t>(k1) << LOG_N2);
  ci v[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) v[r] = gld(reinterpret_cast<const ci *>(y), row + j + r * M8);
  fft8_group<LOG_N2, (LOG_N2 <= 9)>(v, j, hg, 0, T);
#pragma unroll
  for (int q = 0; q < 8; ++q) store_public(y, row + j + q * M8, v[q]);
}

// Decoupled look-back (Merrill & Garland): tile status word = flag << 2 | bits,
// flag 1: aggregate (G << 1 | P), flag 2: inclusive carry-out.  The word holds
// all the information a reader needs, so relaxed device-scope atomics suffice;
// acquire/release at device scope would also write back or invalidate the
// XCD's L2 on every poll.  A tile is its workgroup's blockIdx.x and tiles of a
// product are consecutive in the grid's x dimension, so every tile looked at
// belongs to a workgroup dispatched earlier, which publishes its aggregate
// before it waits itself: with in-order workgroup dispatch the wait always
// ends.  A generous spin limit turns a hang into a reported error
// (carry_err, SSA_DEVICE_ERROR) should that order ever not hold.
static constexpr uint32_t SPIN_LIMIT = 1u << 22;

__device__ uint32_t lookback(uint32_t *tiles, uint32_t tile, uint32_t G, uint32_t P,
                             unsigned int *err) {
  if (tile == 0) {
    __hip_atomic_store(&tiles[0], (2u << 2) | G, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return 0u;
  }
  __hip_atomic_store(&tiles[tile * TILE_WORD_STRIDE], (1u << 2) | (G << 1) | P, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
  uint32_t cin = 0u;
  int idx = static_cast<int>(tile) - 1;
  uint32_t spins = 0u;
  while (idx >= 0) {
    const uint32_t w =
        __hip_atomic_load(&tiles[idx * TILE_WORD_STRIDE], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t f = w >> 2;
    if (f == 0u) {
      if (++spins > SPIN_LIMIT) {
        atomicAdd(err, 1u);
        break;
      }
      __builtin_amdgcn_s_sleep(4);
      continue;
    }
    if (f == 2u) {
      cin = w & 1u;
      break;
    }
    if ((w >> 1) & 1u) {
      cin = 1u;
      break;
    }
    if (!(w & 1u)) {
      cin = 0u;
      break;
    }
    --idx;  // predecessor propagates: look further back
  }
  __hip_atomic_store(&tiles[tile * TILE_WORD_STRIDE], (2u << 2) | (G | (P & cin)),
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return cin;
}

// grid = (max tiles, tasks), CARRY_THREADS threads, tile = blockIdx.x.  The tile's coefficients
// (with 8 before it) are staged in LDS by coalesced loads first, so the six
// overlapping reads per position hit LDS and each lane issues few global loads.
__device__ __forceinline__ void carry_tile(const task &tk, uint32_t tile, int bits) {
  __shared__ uint32_t sh_waves[CARRY_THREADS / 64];
  __shared__ unsigned long long sC[CARRY_TILE + 8];
  const bool failed = (tk.st->too_wide + tk.st->internal) != 0u;
  const long long p0 = static_cast<long long>(tile) * CARRY_TILE;
  const long long base = p0 - 8;
  const uint32_t nout = tk.na + tk.nb;
  const unsigned long long *c = tk.c;
  const long long L = tk.L;
  // Every load of a thread is issued before the first is waited for: PER
  // independent loads in flight per lane instead of one round trip each.
  constexpr int PER = (CARRY_TILE + 8 + CARRY_THREADS - 1) / CARRY_THREADS;
  unsigned long long lo[PER], hi[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int t = threadIdx.x + k * CARRY_THREADS;
    const long long q = base + t;
    const bool in = t < CARRY_TILE + 8 && q >= 0;
    if (bits == 8) {
      lo[k] = (in && q < L) ? gload(c + q) : 0ull;
      hi[k] = 0ull;
    } else {
      lo[k] = (in && 2 * q < L) ? gload(c + 2 * q) : 0ull;
      hi[k] = (in && 2 * q + 1 < L) ? gload(c + 2 * q + 1) : 0ull;
    }
  }
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int t = threadIdx.x + k * CARRY_THREADS;
    if (t < CARRY_TILE + 8) sC[t] = lo[k] + 16ull * hi[k];
  }
  __syncthreads();
  auto C = [&](long long q) -> unsigned long long { return sC[q - base]; };
  auto tc = [&](uint32_t G, uint32_t P) { return lookback(tk.tiles, tile, G, P, &tk.st->carry_err); };
  carry_block<CARRY_CHUNKS>(C, p0, nout, tk.out, failed, tc, sh_waves);
}

// grid = (max tiles, tasks); workgroups past a product's last tile exit at once.
__global__ __launch_bounds__(CARRY_THREADS) void k_carry(const task *tasks, int bits) {
  const task tk = tasks[gridDim.y - 1 - blockIdx.y];  // last written first
  const uint32_t tile = blockIdx.x;
  if (tile >= tk.ntiles) return;
  carry_tile(tk, tile, bits);
}

// grid = (number of tiles): workgroup x takes tile map[x].y of task map[x].x.
// The map lists every tile of every product once, each product's tiles
// consecutive and in increasing order (the look-back's dispatch order), so
// products of uneven lengths launch no idle workgroups.
__global__ __launch_bounds__(CARRY_THREADS) void k_carry_map(const task *tasks, const uint2 *map,
                                                            int bits) {
  const uint2 m = map[blockIdx.x];
  carry_tile(tasks[m.x], m.y, bits);
}

// Final status per product: 0 ok, 1 too wide, 4 device error, 5 internal.
__global__ void k_status(const task *tasks, int ntasks, int *status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ntasks) return;
  const dev_stats *st = tasks[i].st;
  int s = 0;
  if (st->internal) s = 5;
  else if (st->too_wide) s = 1;
  else if (st->carry_err) s = 4;
  status[i] = s;
}

// Directed-rounding probe: the primitives above on n inputs.
// op 0: RU(a+b)  1: RU(a*b)  2: RU(a*b+c)  3: RD(a+b)  4: RD(a*b)  5: RD(a*b+c)
__global__ void k_probe(int op, const double *a, const double *b, const double *c, double *out,
                        size_t n) {
  const uint32_t z = enter_round_up();
  a = after_mode(a, z);
  const size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  const double x = a[i], y = b[i], w = c[i];
  double r;
  switch (op) {
    case 0: r = ru_add(x, y); break;
    case 1: r = ru_mul(x, y); break;
    case 2: r = ru_fma(x, y, w); break;
    case 3: r = -ru_add(-x, -y); break;
    case 4: r = -ru_nmul(x, y); break;
    default: r = -ru_fma(-x, y, -w); break;
  }
  out[i] = r;
}

// Certification of caller-supplied enclosures, one per thread: the same
// certify() and cert_reduce() as the product kernels.  cls[i] (when given) is
// the entry's outcome, 0 one integer, 1 several, 5 impossible, plus 16 when
// the real part contains a half-integer.
__global__ __launch_bounds__(256) void k_certify_probe(const double *enc, uint32_t n, uint32_t L,
                                                       int mode, unsigned long long *c, int *cls,
                                                       dev_stats *st) {
  __shared__ cert_shared sh;
  const uint32_t z = enter_round_up();
  enc = after_mode(enc, z);
  if (threadIdx.x == 0) sh = cert_shared{0ull, 0ull, 0u, 0u};
  __syncthreads();
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  cert_acc acc{0.0, 0u, 0u, 0u};
  if (i < n) {
    const ci e = gld(reinterpret_cast<const ci *>(enc), i);  // {re_lo, re_hi, im_lo, im_hi}
    const ci v{-e.rn, e.rh, -e.in, e.ih};
    const unsigned long long cv = certify(v, i, L, mode, acc);
    if (i < L) c[i] = cv;
    if (cls != nullptr)
      cls[i] = (acc.internal ? 5 : (acc.too_wide ? 1 : 0)) | (acc.half ? 16 : 0);
  }
  cert_reduce(sh, acc);
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicMax(&st->max_rad_bits, sh.rad_bits);
    if (sh.half) atomicAdd(&st->half_int, sh.half);
    if (sh.too_wide) atomicAdd(&st->too_wide, sh.too_wide);
    if (sh.internal) atomicAdd(&st->internal, sh.internal);
  }
}

// Statuses from batch slot order back to the caller's order.
__global__ void k_scatter(const int *slot_status, const int *order, int n, int *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[order[i]] = slot_status[i];
}

// ---------------------------------------------------------------------------
// Host launchers.

static constexpr int MAX_DYN_LDS = 131072;

// Kernels are instantiated per transform length: k_small for 2^9..2^12, the
// column and row passes for column / row lengths 2^6..2^11.  These switches
// map a run-time length to its instantiation (F is a macro taking the length).
#define SSA_SMALL_LENGTHS(F) F(9) F(10) F(11) F(12)
#define SSA_PASS_LENGTHS(F) F(6) F(7) F(8) F(9) F(10) F(11)
#define SSA_ROW_PERSIST_LENGTHS(F) F(6) F(7) F(8) F(9)

hipError_t set_kernel_attributes() {
  const void *ks[] = {
#define SSA_K_SMALL(L)                                                                      \
  reinterpret_cast<const void *>(&k_small<L, 8, 1, ci>), reinterpret_cast<const void *>(&k_small<L, 4, 1, ci>), \
      reinterpret_cast<const void *>(&k_small<L, 8, 0, ci>), reinterpret_cast<const void *>(&k_small<L, 4, 0, ci>), \
      reinterpret_cast<const void *>(&k_small<L, 8, 1, md>), reinterpret_cast<const void *>(&k_small<L, 4, 1, md>), \
      reinterpret_cast<const void *>(&k_small<L, 8, 1, pt>), reinterpret_cast<const void *>(&k_small<L, 4, 1, pt>), \
      reinterpret_cast<const void *>(&k_small<L, 8, 1, pf>), reinterpret_cast<const void *>(&k_small<L, 4, 1, pf>),
      SSA_SMALL_LENGTHS(SSA_K_SMALL)
#undef SSA_K_SMALL
#define SSA_K_PASS(L)                                                                    \
  reinterpret_cast<const void *>(&k_col_fwd<L, 1, 8, ci>), reinterpret_cast<const void *>(&k_col_fwd<L, 1, 4, ci>), \
      reinterpret_cast<const void *>(&k_col_fwd<L, 0, 8, ci>), reinterpret_cast<const void *>(&k_col_fwd<L, 0, 4, ci>), \
      reinterpret_cast<const void *>(&k_col_fwd<L, 1, 8, md>), reinterpret_cast<const void *>(&k_col_fwd<L, 1, 4, md>), \
      reinterpret_cast<const void *>(&k_col_fwd<L, 1, 8, pt>), reinterpret_cast<const void *>(&k_col_fwd<L, 1, 4, pt>), \
      reinterpret_cast<const void *>(&k_row<L>), \
      reinterpret_cast<const void *>(&k_row_pair<L, ci>), reinterpret_cast<const void *>(&k_col_inv<L, ci>), \
      reinterpret_cast<const void *>(&k_row_pair<L, md>), reinterpret_cast<const void *>(&k_col_inv<L, md>), \
      reinterpret_cast<const void *>(&k_row_pair<L, pt>), reinterpret_cast<const void *>(&k_col_inv<L, pt>), \
      reinterpret_cast<const void *>(&k_fft_col<L>), reinterpret_cast<const void *>(&k_fft_row<L>),
      SSA_PASS_LENGTHS(SSA_K_PASS)
#undef SSA_K_PASS
#define SSA_K_ROWP(L) reinterpret_cast<const void *>(&k_row_pair_p<L>),
      SSA_ROW_PERSIST_LENGTHS(SSA_K_ROWP)
#undef SSA_K_ROWP
  };
  for (const void *k : ks) {
    const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, MAX_DYN_LDS);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_scatter_status(const int *slot_status, const int *order, int n, int *out,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_scatter, dim3((n + 255) / 256), dim3(256), 0, s, slot_status, order, n, out);
  return hipGetLastError();
}

static twtab to_dev(const twtab_host &t) { return twtab{t.tab, t.log_ntab, t.e}; }

static inline void mark(const timing_hook *hk, int kind, int phase) {
  if (hk != nullptr) hk->mark(hk->ctx, kind, phase);
}

hipError_t launch_small(const task *d_tasks, int ntasks, int log_n, int digit_bits, int cert_mode,
                        int pack, int arith, int fp32, int rerun, int hooks, const twtab_host &tw,
                        double *dbg, hipStream_t s, const timing_hook *hk) {
  const int threads = 1 << (log_n - 3);
  const size_t lds = sizeof(double2) * lpad_size(size_t(1) << log_n);
  if (arith != ARITH_RECT && !pack) return hipErrorInvalidValue;  // discs, points: packed only
  if ((arith == ARITH_POINT || arith == ARITH_POINT32) && fp32) return hipErrorInvalidValue;
  mark(hk, KIND_SMALL, 0);
  switch (log_n) {
#define SSA_L(L)                                                                               \
  case L:                                                                                      \
    if (arith == ARITH_DISC && digit_bits == 8)                                                 \
      hipLaunchKernelGGL((k_small<L, 8, 1, md>), dim3(ntasks), dim3(threads), lds, s, d_tasks,  \
                         cert_mode, fp32, rerun, hooks, to_dev(tw), dbg);                       \
    else if (arith == ARITH_DISC)                                                               \
      hipLaunchKernelGGL((k_small<L, 4, 1, md>), dim3(ntasks), dim3(threads), lds, s, d_tasks,  \
                         cert_mode, fp32, rerun, hooks, to_dev(tw), dbg);                       \
    else if (arith == ARITH_POINT && digit_bits == 8)                                           \
      hipLaunchKernelGGL((k_small<L, 8, 1, pt>), dim3(ntasks), dim3(threads), lds, s, d_tasks,  \
                         cert_mode, fp32, rerun, hooks, to_dev(tw), dbg);                       \
    else if (arith == ARITH_POINT)                                                              \
      hipLaunchKernelGGL((k_small<L, 4, 1, pt>), dim3(ntasks), dim3(threads), lds, s, d_tasks,  \
                         cert_mode, fp32, rerun, hooks, to_dev(tw), dbg);                       \
    else if (arith == ARITH_POINT32 && digit_bits == 8)                                         \
      hipLaunchKernelGGL((k_small<L, 8, 1, pf>), dim3(ntasks), dim3(threads), lds, s, d_tasks,  \
                         cert_mode, fp32, rerun, hooks, to_dev(tw), dbg);                       \
    else if (arith == ARITH_POINT32)                                                            \
      hipLaunchKernelGGL((k_small<L, 4, 1, pf>), dim3(ntasks), dim3(threads), lds, s, d_tasks,  \
                         cert_mode, fp32, rerun, hooks, to_dev(tw), dbg);                       \
    else if (digit_bits == 8 && pack)                                                           \
      hipLaunchKernelGGL((k_small<L, 8, 1, ci>), dim3(ntasks), dim3(threads), lds, s, d_tasks,  \
                         cert_mode, fp32, rerun, hooks, to_dev(tw), dbg);                       \
    else if (pack)                                                                              \
      hipLaunchKernelGGL((k_small<L, 4, 1, ci>), dim3(ntasks), dim3(threads), lds, s, d_tasks,  \
                         cert_mode, fp32, rerun, hooks, to_dev(tw), dbg);                       \
    else if (digit_bits == 8)                                                                   \
      hipLaunchKernelGGL((k_small<L, 8, 0, ci>), dim3(ntasks), dim3(threads), lds, s, d_tasks,  \
                         cert_mode, fp32, rerun, hooks, to_dev(tw), dbg);                       \
    else                                                                                        \
      hipLaunchKernelGGL((k_small<L, 4, 0, ci>), dim3(ntasks), dim3(threads), lds, s, d_tasks,  \
                         cert_mode, fp32, rerun, hooks, to_dev(tw), dbg);                       \
    break;
    SSA_SMALL_LENGTHS(SSA_L)
#undef SSA_L
    default:
      return hipErrorInvalidValue;
  }
  mark(hk, KIND_SMALL, 1);
  return hipGetLastError();
}

// Workgroups of a kernel resident at once on the whole GPU (occupancy per CU
// times CUs), cached per kernel and shape; at least 1.
static uint32_t resident_workgroups(const void *kernel, int threads, size_t lds) {
  struct entry {
    const void *k;
    int t;
    size_t l;
    uint32_t n;
  };
  static entry cache[64];
  static int used = 0;
  for (int i = 0; i < used; ++i)
    if (cache[i].k == kernel && cache[i].t == threads && cache[i].l == lds) return cache[i].n;
  int per_cu = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds) != hipSuccess ||
      hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    (void)hipGetLastError();
    per_cu = 1;
    cus = 1;
  }
  const uint32_t n = static_cast<uint32_t>(std::max(1, per_cu) * std::max(1, cus));
  if (used < 64) cache[used++] = entry{kernel, threads, lds, n};
  return n;
}

static inline int log2_int(int x) {
  int l = 0;
  while ((1 << l) < x) ++l;
  return l;
}

hipError_t launch_multipass(const task *d_tasks, int ntasks, int log_n, const launch_cfg &cfg,
                            int digit_bits, int cert_mode, const twtab_host &tw, double *dbg,
                            hipStream_t s, const timing_hook *hk) {
  const int l1 = cfg.log_n1, l2 = cfg.log_n2;
  const uint32_t N1 = 1u << l1, N2 = 1u << l2;
  const int lc = log2_int(cfg.cols);
  const twtab T = to_dev(tw);
  if (l1 < 6 || l1 > 11 || l2 < 6 || l2 > 11 || (1 << lc) != cfg.cols) return hipErrorInvalidValue;
  if (cfg.arith != ARITH_RECT && (!cfg.pack || cfg.persist))
    return hipErrorInvalidValue;  // discs and points: packed transform, plain row pass
  if (cfg.arith == ARITH_POINT32) return hipErrorInvalidValue;  // single-workgroup lengths only
  {
    const int threads = cfg.cols * static_cast<int>(N1 / 8);
    const size_t lds = sizeof(double2) * lpad_size(N1) * cfg.cols;
    const dim3 grid(N2 / cfg.cols, cfg.pack ? 1 : 2, ntasks);
    mark(hk, KIND_COL_FWD, 0);
    switch (l1) {
#define SSA_L(L)                                                                                     \
  case L:                                                                                            \
    if (cfg.arith == ARITH_DISC && digit_bits == 8)                                                  \
      hipLaunchKernelGGL((k_col_fwd<L, 1, 8, md>), grid, dim3(threads), lds, s, d_tasks, l2, lc, T);  \
    else if (cfg.arith == ARITH_DISC)                                                                \
      hipLaunchKernelGGL((k_col_fwd<L, 1, 4, md>), grid, dim3(threads), lds, s, d_tasks, l2, lc, T);  \
    else if (cfg.arith == ARITH_POINT && digit_bits == 8)                                            \
      hipLaunchKernelGGL((k_col_fwd<L, 1, 8, pt>), grid, dim3(threads), lds, s, d_tasks, l2, lc, T);  \
    else if (cfg.arith == ARITH_POINT)                                                               \
      hipLaunchKernelGGL((k_col_fwd<L, 1, 4, pt>), grid, dim3(threads), lds, s, d_tasks, l2, lc, T);  \
    else if (cfg.pack && digit_bits == 8)                                                            \
      hipLaunchKernelGGL((k_col_fwd<L, 1, 8, ci>), grid, dim3(threads), lds, s, d_tasks, l2, lc, T);  \
    else if (cfg.pack)                                                                               \
      hipLaunchKernelGGL((k_col_fwd<L, 1, 4, ci>), grid, dim3(threads), lds, s, d_tasks, l2, lc, T);  \
    else if (digit_bits == 8)                                                                        \
      hipLaunchKernelGGL((k_col_fwd<L, 0, 8, ci>), grid, dim3(threads), lds, s, d_tasks, l2, lc, T);  \
    else                                                                                             \
      hipLaunchKernelGGL((k_col_fwd<L, 0, 4, ci>), grid, dim3(threads), lds, s, d_tasks, l2, lc, T);  \
    break;
      SSA_PASS_LENGTHS(SSA_L)
#undef SSA_L
    }
    mark(hk, KIND_COL_FWD, 1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (cfg.pack && cfg.persist) {
    const int threads = 2 * cfg.rows * static_cast<int>(N2 / 8);
    const size_t lds = sizeof(double2) * (2 * lpad_size(N2) * cfg.rows + (size_t(2) << l2));
    const uint32_t total = N1 / 2 / cfg.rows * static_cast<uint32_t>(ntasks);
    mark(hk, KIND_ROW, 0);
    switch (l2) {
#define SSA_L(L)                                                                                  \
  case L: {                                                                                       \
    const uint32_t res = resident_workgroups(reinterpret_cast<const void *>(&k_row_pair_p<L>),    \
                                             threads, lds);                                       \
    hipLaunchKernelGGL(k_row_pair_p<L>, dim3(std::min(total, res)), dim3(threads), lds, s,        \
                       d_tasks, ntasks, l1, cfg.rows, T);                                         \
    break;                                                                                        \
  }
      SSA_ROW_PERSIST_LENGTHS(SSA_L)
#undef SSA_L
      default:
        return hipErrorInvalidValue;
    }
    mark(hk, KIND_ROW, 1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  } else if (cfg.pack) {
    const int threads = 2 * cfg.rows * static_cast<int>(N2 / 8);
    const size_t lds = sizeof(double2) * 2 * lpad_size(N2) * cfg.rows;
    const dim3 grid(N1 / 2 / cfg.rows, ntasks);
    mark(hk, KIND_ROW, 0);
    switch (l2) {
#define SSA_L(L)                                                                                    \
  case L:                                                                                           \
    if (cfg.arith == ARITH_DISC)                                                                    \
      hipLaunchKernelGGL((k_row_pair<L, md>), grid, dim3(threads), lds, s, d_tasks, l1, cfg.rows, T); \
    else if (cfg.arith == ARITH_POINT)                                                              \
      hipLaunchKernelGGL((k_row_pair<L, pt>), grid, dim3(threads), lds, s, d_tasks, l1, cfg.rows, T); \
    else                                                                                            \
      hipLaunchKernelGGL((k_row_pair<L, ci>), grid, dim3(threads), lds, s, d_tasks, l1, cfg.rows, T); \
    break;
      SSA_PASS_LENGTHS(SSA_L)
#undef SSA_L
    }
    mark(hk, KIND_ROW, 1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  } else {
    const int threads = cfg.rows * static_cast<int>(N2 / 8);
    const size_t lds = sizeof(double2) * lpad_size(N2) * cfg.rows;
    const dim3 grid(N1 / cfg.rows, ntasks);
    mark(hk, KIND_ROW, 0);
    switch (l2) {
#define SSA_L(L)                                                                               \
  case L:                                                                                      \
    hipLaunchKernelGGL(k_row<L>, grid, dim3(threads), lds, s, d_tasks, l1, cfg.rows, T);      \
    break;
      SSA_PASS_LENGTHS(SSA_L)
#undef SSA_L
    }
    mark(hk, KIND_ROW, 1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  {
    const int lci = log2_int(cfg.icols);
    if ((1 << lci) != cfg.icols) return hipErrorInvalidValue;
    const int threads = cfg.icols * static_cast<int>(N1 / 8);
    const size_t lds = sizeof(double2) * lpad_size(N1) * cfg.icols;
    const dim3 grid(N2 / 2 / cfg.icols, ntasks);
    mark(hk, KIND_COL_INV, 0);
    switch (l1) {
#define SSA_L(L)                                                                                \
  case L:                                                                                       \
    if (cfg.arith == ARITH_DISC)                                                                \
      hipLaunchKernelGGL((k_col_inv<L, md>), grid, dim3(threads), lds, s, d_tasks, l2, lci,    \
                         cert_mode, T, dbg);                                                    \
    else if (cfg.arith == ARITH_POINT)                                                          \
      hipLaunchKernelGGL((k_col_inv<L, pt>), grid, dim3(threads), lds, s, d_tasks, l2, lci,    \
                         cert_mode, T, dbg);                                                    \
    else                                                                                        \
      hipLaunchKernelGGL((k_col_inv<L, ci>), grid, dim3(threads), lds, s, d_tasks, l2, lci,    \
                         cert_mode, T, dbg);                                                    \
    break;
      SSA_PASS_LENGTHS(SSA_L)
#undef SSA_L
    }
    mark(hk, KIND_COL_INV, 1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  (void)log_n;
  return hipSuccess;
}

hipError_t launch_fft_forward(const double *x, double *y, int count, const launch_cfg &cfg,
                              const twtab_host &tw, hipStream_t s, hipEvent_t *ev) {
  const int l1 = cfg.log_n1, l2 = cfg.log_n2;
  const uint32_t N1 = 1u << l1, N2 = 1u << l2;
  const int lc = log2_int(cfg.cols);
  const twtab T = to_dev(tw);
  if (l1 < 6 || l1 > 11 || l2 < 6 || l2 > 11 || (1 << lc) != cfg.cols || count < 1 || count > 65535)
    return hipErrorInvalidValue;
  if (ev) (void)hipEventRecord(ev[0], s);
  {
    const int threads = cfg.cols * static_cast<int>(N1 / 8);
    const size_t lds = sizeof(double2) * lpad_size(N1) * cfg.cols;
    const dim3 grid(N2 / cfg.cols, count);
    switch (l1) {
#define SSA_L(L)                                                                                \
  case L:                                                                                       \
    hipLaunchKernelGGL(k_fft_col<L>, grid, dim3(threads), lds, s, x, y, l2, lc, T);            \
    break;
      SSA_PASS_LENGTHS(SSA_L)
#undef SSA_L
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (ev) (void)hipEventRecord(ev[1], s);
  {
    const int threads = cfg.rows * static_cast<int>(N2 / 8);
    const size_t lds = sizeof(double2) * lpad_size(N2) * cfg.rows;
    const dim3 grid(N1 / cfg.rows, count);
    switch (l2) {
#define SSA_L(L)                                                                                \
  case L:                                                                                       \
    hipLaunchKernelGGL(k_fft_row<L>, grid, dim3(threads), lds, s, y, l1, cfg.rows, T);         \
    break;
      SSA_PASS_LENGTHS(SSA_L)
#undef SSA_L
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (ev) (void)hipEventRecord(ev[2], s);
  return hipSuccess;
}

hipError_t launch_carry(const task *d_tasks, int ntasks, uint32_t max_tiles, int digit_bits,
                        hipStream_t s, const timing_hook *hk) {
  mark(hk, KIND_CARRY, 0);
  hipLaunchKernelGGL(k_carry, dim3(max_tiles, ntasks), dim3(CARRY_THREADS), 0, s, d_tasks,
                     digit_bits);
  mark(hk, KIND_CARRY, 1);
  return hipGetLastError();
}

hipError_t launch_carry_map(const task *d_tasks, const uint2 *d_map, uint32_t ntiles,
                            int digit_bits, hipStream_t s, const timing_hook *hk) {
  mark(hk, KIND_CARRY, 0);
  hipLaunchKernelGGL(k_carry_map, dim3(ntiles), dim3(CARRY_THREADS), 0, s, d_tasks, d_map,
                     digit_bits);
  mark(hk, KIND_CARRY, 1);
  return hipGetLastError();
}

hipError_t launch_status(const task *d_tasks, int ntasks, int *d_status, hipStream_t s,
                         const timing_hook *hk) {
  mark(hk, KIND_STATUS, 0);
  hipLaunchKernelGGL(k_status, dim3((ntasks + 255) / 256), dim3(256), 0, s, d_tasks, ntasks,
                     d_status);
  mark(hk, KIND_STATUS, 1);
  return hipGetLastError();
}

hipError_t launch_certify_probe(const double *enc, uint32_t n, uint32_t L, int mode,
                                unsigned long long *c, int *cls, dev_stats *st, hipStream_t s) {
  hipLaunchKernelGGL(k_certify_probe, dim3((n + 255) / 256), dim3(256), 0, s, enc, n, L, mode, c,
                     cls, st);
  return hipGetLastError();
}

hipError_t launch_directed_probe(int op, const double *a, const double *b, const double *c,
                                 double *out, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_probe, dim3((n + 255) / 256), dim3(256), 0, s, op, a, b, c, out, n);
  return hipGetLastError();
}

}  // namespace ssa
