// CPU ORACLE for rigorous complex-interval Schoenhage-Strassen multiplication.
//
// This file is TEST INFRASTRUCTURE.  It is a plain, slow, single-threaded
// restatement of the paper's method (Steinke & Sainudiin, "A Rigorous Extension
// of the Schoenhage-Strassen Integer Multiplication Algorithm Using Complex
// Interval Arithmetic", CCA 2010) written for checking the GPU library against.
// Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
// load it.  It shares no code, header, table or helper with the GPU library.
//
// Arithmetic: only IEEE + - * / sqrt, each evaluated under fesetround() with the
// direction the interval bound needs (lower bounds toward -inf, upper bounds
// toward +inf).  No libm transcendental function is used anywhere.  Build with
// -frounding-math -fno-fast-math -ffp-contract=off so the compiler neither folds
// nor fuses across rounding-mode changes; every directed operation is also a
// noinline function whose operands pass through an opaque barrier after the mode
// switch, so no operation can be scheduled under the wrong mode.
//
// Structure (paper section 2):
//   * integer digit vectors, little-endian, base b (section 2, start);
//   * real intervals IR with + - * / and sqrt, rectangular complex intervals IC
//     with +, -, * and division by a positive integer (section 2.5);
//   * the primitive roots from the half-angle recurrence (section 2.2, closing
//     remark on computing omega), powers of omega as products over the set bits
//     of the exponent;
//   * the recursive radix-2 Cooley-Tukey FFT (section 2.2, FFT box);
//   * fast convolution (section 2.3, Fast Convolution box);
//   * certification: take the unique integer in each enclosure or report an
//     error (section 1, paragraph on containment sets; section 2.5);
//   * carries (section 2.4, SSA box).
//
// Parity pins (tests under tests/): schoolbook long multiplication, the CPython
// integer product, all-0xFF closed forms, hand-worked tiny products, DFT special
// cases from the Lemma of section 2.2, twiddles against mpmath interval
// arithmetic, directed-rounding primitives against exact rationals.  Enclosure
// radii and the certification frontier are "parity unpinned": the paper prints
// no values for them.

#include <cfenv>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <cstddef>
#include <vector>
#include <algorithm>


namespace {

// ---------------------------------------------------------------------------
// Status codes (same numeric meaning as the library's public status codes, but
// defined independently here).
enum { ST_OK = 0, ST_TOO_WIDE = 1, ST_INVALID = 2, ST_INTERNAL = 5 };

// Planted-mistake switch, used ONLY by the tests that check the pins are able
// to catch a wrong oracle.  0 = the correct method.  Every other value plants
// one plausible mistake at one place (listed next to the place).
int g_mutation = 0;

#define NOINLINE __attribute__((noinline))

// Opaque barrier: after a rounding-mode switch, the operands "change" as far as
// the compiler knows, so the arithmetic that follows cannot be hoisted above it.
template <class T> inline void opaque(T &x) { __asm__ volatile("" : "+m"(x)); }

// ---------------------------------------------------------------------------
// Directed-rounding scalar operations.  Each sets the mode, computes, restores
// round-to-nearest.

template <class T> NOINLINE T add_dir(T a, T b, int mode) {
  std::fesetround(mode); opaque(a); opaque(b);
  T r = a + b; opaque(r);
  std::fesetround(FE_TONEAREST);
  return r;
}
template <class T> NOINLINE T sub_dir(T a, T b, int mode) {
  std::fesetround(mode); opaque(a); opaque(b);
  T r = a - b; opaque(r);
  std::fesetround(FE_TONEAREST);
  return r;
}
template <class T> NOINLINE T mul_dir(T a, T b, int mode) {
  std::fesetround(mode); opaque(a); opaque(b);
  T r = a * b; opaque(r);
  std::fesetround(FE_TONEAREST);
  return r;
}
template <class T> NOINLINE T div_dir(T a, T b, int mode) {
  std::fesetround(mode); opaque(a); opaque(b);
  T r = a / b; opaque(r);
  std::fesetround(FE_TONEAREST);
  return r;
}
template <class T> NOINLINE T sqrt_dir(T a, int mode) {
  std::fesetround(mode); opaque(a);
  T r = std::sqrt(a); opaque(r);
  std::fesetround(FE_TONEAREST);
  return r;
}

// ---------------------------------------------------------------------------
// Real intervals IR (section 2.5).  [lo, hi], lo <= hi, closed.

template <class T> struct I { T lo, hi; };

template <class T> I<T> thin(T v) { return I<T>{v, v}; }

// Sum: lower bounds added rounding down, upper bounds rounding up.
template <class T> I<T> iadd(I<T> a, I<T> b) {
  return I<T>{add_dir(a.lo, b.lo, FE_DOWNWARD), add_dir(a.hi, b.hi, FE_UPWARD)};
}
// Difference: [a.lo - b.hi, a.hi - b.lo].
template <class T> I<T> isub(I<T> a, I<T> b) {
  return I<T>{sub_dir(a.lo, b.hi, FE_DOWNWARD), sub_dir(a.hi, b.lo, FE_UPWARD)};
}
// Product: min of the four end-point products rounded down, max of the four
// rounded up.
template <class T> I<T> imul(I<T> a, I<T> b) {
  T l1 = mul_dir(a.lo, b.lo, FE_DOWNWARD), l2 = mul_dir(a.lo, b.hi, FE_DOWNWARD);
  T l3 = mul_dir(a.hi, b.lo, FE_DOWNWARD), l4 = mul_dir(a.hi, b.hi, FE_DOWNWARD);
  T h1 = mul_dir(a.lo, b.lo, FE_UPWARD), h2 = mul_dir(a.lo, b.hi, FE_UPWARD);
  T h3 = mul_dir(a.hi, b.lo, FE_UPWARD), h4 = mul_dir(a.hi, b.hi, FE_UPWARD);
  if (g_mutation == 4) {  // planted: lower bound rounded to nearest
    l1 = a.lo * b.lo; l2 = a.lo * b.hi; l3 = a.hi * b.lo; l4 = a.hi * b.hi;
  }
  return I<T>{std::min(std::min(l1, l2), std::min(l3, l4)),
              std::max(std::max(h1, h2), std::max(h3, h4))};
}
// Quotient by an interval not containing 0: a * [1/b.hi, 1/b.lo], here
// evaluated as the min/max of the four end-point quotients with directed
// rounding (one rounding per bound instead of two, the same containment).
template <class T> bool idiv(I<T> a, I<T> b, I<T> *r) {
  if (b.lo <= 0 && b.hi >= 0) return false;  // undefined when 0 is in b
  T l1 = div_dir(a.lo, b.lo, FE_DOWNWARD), l2 = div_dir(a.lo, b.hi, FE_DOWNWARD);
  T l3 = div_dir(a.hi, b.lo, FE_DOWNWARD), l4 = div_dir(a.hi, b.hi, FE_DOWNWARD);
  T h1 = div_dir(a.lo, b.lo, FE_UPWARD), h2 = div_dir(a.lo, b.hi, FE_UPWARD);
  T h3 = div_dir(a.hi, b.lo, FE_UPWARD), h4 = div_dir(a.hi, b.hi, FE_UPWARD);
  r->lo = std::min(std::min(l1, l2), std::min(l3, l4));
  r->hi = std::max(std::max(h1, h2), std::max(h3, h4));
  return true;
}
// Square root on a non-negative interval: [sqrt(lo), sqrt(hi)].
template <class T> bool isqrt(I<T> a, I<T> *r) {
  if (a.lo < 0) return false;
  r->lo = sqrt_dir(a.lo, FE_DOWNWARD);
  r->hi = sqrt_dir(a.hi, FE_UPWARD);
  return true;
}

// ---------------------------------------------------------------------------
// Rectangular complex intervals IC (section 2.5): [z1] + i[z2].

template <class T> struct C { I<T> re, im; };

template <class T> C<T> cadd(const C<T> &a, const C<T> &b) {
  return C<T>{iadd(a.re, b.re), iadd(a.im, b.im)};
}
template <class T> C<T> csub(const C<T> &a, const C<T> &b) {
  return C<T>{isub(a.re, b.re), isub(a.im, b.im)};
}
// Product: ([z1][w1] - [z2][w2]) + i([z1][w2] + [z2][w1]).
template <class T> C<T> cmul(const C<T> &z, const C<T> &w) {
  if (g_mutation == 3)  // planted: operands of the real part swapped
    return C<T>{isub(imul(z.re, w.re), imul(z.re, w.im)),
                iadd(imul(z.re, w.im), imul(z.im, w.re))};
  return C<T>{isub(imul(z.re, w.re), imul(z.im, w.im)),
              iadd(imul(z.re, w.im), imul(z.im, w.re))};
}
// Division by a positive integer n, componentwise.
template <class T> C<T> cdiv_int(const C<T> &z, uint64_t n) {
  I<T> d = thin(static_cast<T>(n));  // n = 2^k is exactly representable
  C<T> r;
  idiv(z.re, d, &r.re);
  idiv(z.im, d, &r.im);
  return r;
}
// Conjugate: exact negation of the imaginary bounds.
template <class T> C<T> conj(const C<T> &z) {
  return C<T>{z.re, I<T>{-z.im.hi, -z.im.lo}};
}

// ---------------------------------------------------------------------------
// Primitive roots omega_{2^s} = e^{2 pi i / 2^s} from the half-angle
// recurrence of section 2.2:  omega_1 = 1, omega_2 = -1, omega_4 = i and
// omega_{2n} = (1 + omega_n) / |1 + omega_n| for n >= 4 (the recurrence is
// stated for n >= 3; over powers of two that means n >= 4, since n = 2 would
// divide by |1 + (-1)| = 0).  R[s] encloses omega_{2^s}.
template <class T> std::vector<C<T>> roots(int k) {
  std::vector<C<T>> R(static_cast<size_t>(std::max(k, 2)) + 1);
  R[0] = C<T>{thin<T>(1), thin<T>(0)};
  R[1] = C<T>{thin<T>(-1), thin<T>(0)};
  R[2] = C<T>{thin<T>(0), thin<T>(1)};
  for (int s = 2; s < k; ++s) {
    C<T> num{iadd(thin<T>(1), R[s].re), R[s].im};      // 1 + omega_n
    I<T> sq = iadd(imul(num.re, num.re), imul(num.im, num.im));
    I<T> mag;
    isqrt(sq, &mag);                                    // |1 + omega_n|
    C<T> q;
    idiv(num.re, mag, &q.re);
    idiv(num.im, mag, &q.im);
    R[s + 1] = q;
  }
  R.resize(static_cast<size_t>(k) + 1);
  return R;
}

// Powers omega_N^j, 0 <= j < N/2, N = 2^k.  The paper does not say how the
// powers in the FFT box are formed; this oracle multiplies together the roots
// for the set bits of j: omega_N^{2^t} = omega_{2^{k-t}} = R[k-t], and
// T[j] = T[j - 2^t] * R[k-t] with t the highest set bit of j.
template <class T> std::vector<C<T>> twiddles(int k) {
  size_t N = size_t(1) << k;
  size_t half = N / 2;
  std::vector<C<T>> Tw(std::max<size_t>(half, 1));
  Tw[0] = C<T>{thin<T>(1), thin<T>(0)};
  if (k == 0) return Tw;
  std::vector<C<T>> R = roots<T>(k);
  for (size_t j = 1; j < half; ++j) {
    int t = 63 - __builtin_clzll(static_cast<unsigned long long>(j));
    size_t rest = j - (size_t(1) << t);
    int root = k - t;
    if (g_mutation == 7) root = k - t - 1;  // planted: off-by-one root index
    Tw[j] = cmul(Tw[rest], R[root]);
  }
  return Tw;
}

// ---------------------------------------------------------------------------
// The Cooley-Tukey FFT box (section 2.2): recursive, radix 2.  x has 2^k
// entries; Tw is the table for the top-level length Ntop = 2^ktop, and the
// length-M sub-transform uses omega_M^i = Tw[i * Ntop / M].  The combine step
// is written with the symmetric pair  X_i = E_i + w O_i,  X_{i+M/2} = E_i - w O_i,
// which equals the box's  X_i = E_{i mod M/2} + omega^i O_{i mod M/2}  because
// omega^{i+M/2} = -omega^i and interval negation is exact.  For the inverse
// transform the twiddles are conjugated (omega^{-1} = conj omega).
template <class T>
std::vector<C<T>> fft_rec(int k, const std::vector<C<T>> &x,
                          const std::vector<C<T>> &Tw, int ktop, bool inverse) {
  if (k == 0) return x;                            // the DFT of length 1
  size_t M = size_t(1) << k, H = M / 2;
  std::vector<C<T>> ev(H), od(H);
  for (size_t i = 0; i < H; ++i) { ev[i] = x[2 * i]; od[i] = x[2 * i + 1]; }
  if (g_mutation == 8) std::swap(ev, od);          // planted: even/odd swapped
  std::vector<C<T>> E = fft_rec(k - 1, ev, Tw, ktop, inverse);
  std::vector<C<T>> O = fft_rec(k - 1, od, Tw, ktop, inverse);
  std::vector<C<T>> X(M);
  size_t stride = (size_t(1) << ktop) / M;
  for (size_t i = 0; i < H; ++i) {
    C<T> w = Tw[i * stride];
    if (inverse != (g_mutation == 2)) w = conj(w);  // planted 2: wrong sign
    if (g_mutation == 1) w = C<T>{thin<T>(1), thin<T>(0)};  // planted: no twiddle
    C<T> t = cmul(w, O[i]);
    X[i] = cadd(E[i], t);
    X[i + H] = csub(E[i], t);
  }
  return X;
}

// Forward DFT (omega = e^{+2 pi i / N}) or inverse DFT including the 1/N
// factor (division of a complex interval by a positive integer).
template <class T>
std::vector<C<T>> dft(int k, const std::vector<C<T>> &x, bool inverse) {
  std::vector<C<T>> Tw = twiddles<T>(k);
  std::vector<C<T>> X = fft_rec(k, x, Tw, k, inverse);
  if (inverse && g_mutation != 5) {  // planted 5: the 1/N factor forgotten
    uint64_t N = uint64_t(1) << k;
    for (auto &v : X) v = cdiv_int(v, N);
  }
  return X;
}

// ---------------------------------------------------------------------------
// Digit handling.  Base 256 digits are the bytes themselves; in base 16 each
// byte v becomes the two digits (v & 15, v >> 4), low digit first.
std::vector<uint32_t> to_digits(const uint8_t *p, size_t n, int digit_bits) {
  std::vector<uint32_t> d;
  if (digit_bits == 8) {
    d.assign(p, p + n);
  } else {
    d.resize(2 * n);
    for (size_t i = 0; i < n; ++i) { d[2 * i] = p[i] & 15u; d[2 * i + 1] = p[i] >> 4; }
  }
  return d;
}

int ceil_log2(uint64_t L) {
  int k = 0;
  while ((uint64_t(1) << k) < L) ++k;
  return k;
}

// Fast convolution box (section 2.3): pad both digit vectors with zeros to
// N = 2^k >= L = n + m - 1, two forward FFTs, pointwise product, inverse FFT.
// Returns the enclosures of all N outputs.
template <class T>
std::vector<C<T>> convolve(const std::vector<uint32_t> &x,
                           const std::vector<uint32_t> &y, int *kout) {
  size_t L = x.size() + y.size() - 1;
  int k = ceil_log2(L);
  size_t N = size_t(1) << k;
  std::vector<C<T>> a(N, C<T>{thin<T>(0), thin<T>(0)}), b = a;
  for (size_t i = 0; i < x.size(); ++i) a[i].re = thin(static_cast<T>(x[i]));
  for (size_t i = 0; i < y.size(); ++i) b[i].re = thin(static_cast<T>(y[i]));
  std::vector<C<T>> A = dft(k, a, false), B = dft(k, b, false);
  std::vector<C<T>> P(N);
  for (size_t i = 0; i < N; ++i) P[i] = cmul(A[i], B[i]);
  *kout = k;
  return dft(k, P, true);
}

// Certification (section 1: choose the unique integer in the containment set,
// report an error if it holds several; section 2.5).  For i < L the real part
// must contain exactly one integer: ceil(lo) == floor(hi).  Two ceil(lo) <
// floor(hi) means several integers: "enclosure too wide".  ceil(lo) > floor(hi)
// (no integer), a single integer that is negative, or an imaginary part that
// excludes 0 cannot happen for a rigorous enclosure of a non-negative integer,
// so it is reported as an internal error.  The padded tail i >= L must contain 0 in both parts.
// mode 1 is the stricter variant that also fails any enclosure that contains a
// half-integer.  Also reports max_i RU((hi - lo)/2) over i < L and the number of
// real enclosures that contain a half-integer.
template <class T>
int certify(const std::vector<C<T>> &Z, size_t L, int mode, std::vector<int64_t> *c,
            double *max_radius, int64_t *half_int) {
  int st = ST_OK;
  double rmax = 0;
  int64_t nhalf = 0;
  c->assign(L, 0);
  for (size_t i = 0; i < Z.size(); ++i) {
    const C<T> &z = Z[i];
    bool im0 = z.im.lo <= 0 && z.im.hi >= 0;
    if (i >= L) {
      if (!(z.re.lo <= 0 && z.re.hi >= 0) || !im0) st = ST_INTERNAL;
      continue;
    }
    double lo = z.re.lo, hi = z.re.hi;
    double r = div_dir(sub_dir(hi, lo, FE_UPWARD), 2.0, FE_UPWARD);
    rmax = std::max(rmax, r);
    // half-integers n + 1/2 in [lo, hi]: ceil(lo - 1/2) <= floor(hi - 1/2)
    bool half = std::ceil(sub_dir(lo, 0.5, FE_DOWNWARD)) <= std::floor(sub_dir(hi, 0.5, FE_UPWARD));
    if (half) ++nhalf;
    double m = std::ceil(lo), M = std::floor(hi);
    if (m > M || !im0) { st = ST_INTERNAL; continue; }
    if (m < M || (mode == 1 && half)) { if (st == ST_OK) st = ST_TOO_WIDE; continue; }
    if (m < 0) { st = ST_INTERNAL; continue; }  // the one integer is negative
    (*c)[i] = static_cast<int64_t>(m);
  }
  *max_radius = rmax;
  *half_int = nhalf;
  return st;
}

// Carries (section 2.4, SSA box), in the digit base b = 2^digit_bits:
// z_i = (c_i + carry) mod b, carry = floor((c_i + carry) / b), and the last
// digit is the final carry.  Base-16 digits are then packed two per byte, low
// digit first.  nout = number of output bytes.
void carry(const std::vector<int64_t> &c, int digit_bits, uint8_t *out, size_t nout) {
  uint64_t base = uint64_t(1) << digit_bits;
  std::vector<uint32_t> z(c.size() + 1, 0);
  uint64_t cy = 0;
  for (size_t i = 0; i < c.size(); ++i) {
    uint64_t s = static_cast<uint64_t>(c[i]) + cy;
    z[i] = static_cast<uint32_t>(s % base);
    cy = s / base;
    if (g_mutation == 6) cy = 0;  // planted: carry dropped
  }
  // The last digit is the final carry (for a product it is below b, since the
  // product has n + m digits); larger carries are written out digit by digit.
  z[c.size()] = static_cast<uint32_t>(cy % base);
  for (cy /= base; cy > 0; cy /= base) z.push_back(static_cast<uint32_t>(cy % base));
  std::memset(out, 0, nout);
  if (digit_bits == 8) {
    for (size_t i = 0; i < z.size() && i < nout; ++i) out[i] = static_cast<uint8_t>(z[i]);
  } else {
    for (size_t i = 0; i < z.size() && i / 2 < nout; ++i)
      out[i / 2] |= static_cast<uint8_t>(z[i] << (4 * (i & 1)));
  }
}

template <class T>
int mul_impl(const uint8_t *a, size_t na, const uint8_t *b, size_t nb, int digit_bits,
             int mode, uint8_t *out, double *max_radius, int64_t *half_int) {
  if (!a || !b || !out || na == 0 || nb == 0 || (digit_bits != 8 && digit_bits != 4))
    return ST_INVALID;
  std::vector<uint32_t> x = to_digits(a, na, digit_bits), y = to_digits(b, nb, digit_bits);
  int k = 0;
  std::vector<C<T>> Z = convolve<T>(x, y, &k);
  size_t L = x.size() + y.size() - 1;
  std::vector<int64_t> c;
  double r = 0;
  int64_t h = 0;
  int st = certify(Z, L, mode, &c, &r, &h);
  if (max_radius) *max_radius = r;
  if (half_int) *half_int = h;
  if (st != ST_OK) { std::memset(out, 0, na + nb); return st; }
  carry(c, digit_bits, out, na + nb);
  return ST_OK;
}

// Point (non-interval) FFT in round-to-nearest, the "naive" variant of the
// paper (section 1, single-precision example; section 3, "double naive SS"):
// same recursion, primitive roots from the same recurrence evaluated as plain
// numbers, results rounded to the nearest integer with no guarantee.
template <class T> struct P { T re, im; };

template <class T>
std::vector<P<T>> naive_fft(int k, const std::vector<P<T>> &x, const std::vector<P<T>> &Tw,
                            int ktop, bool inverse) {
  if (k == 0) return x;
  size_t M = size_t(1) << k, H = M / 2;
  std::vector<P<T>> ev(H), od(H);
  for (size_t i = 0; i < H; ++i) { ev[i] = x[2 * i]; od[i] = x[2 * i + 1]; }
  std::vector<P<T>> E = naive_fft(k - 1, ev, Tw, ktop, inverse);
  std::vector<P<T>> O = naive_fft(k - 1, od, Tw, ktop, inverse);
  std::vector<P<T>> X(M);
  size_t stride = (size_t(1) << ktop) / M;
  for (size_t i = 0; i < H; ++i) {
    P<T> w = Tw[i * stride];
    if (inverse && g_mutation != 9) w.im = -w.im;  // planted 9: inverse keeps forward roots
    P<T> t{w.re * O[i].re - w.im * O[i].im, w.re * O[i].im + w.im * O[i].re};
    X[i] = P<T>{E[i].re + t.re, E[i].im + t.im};
    X[i + H] = P<T>{E[i].re - t.re, E[i].im - t.im};
  }
  return X;
}

template <class T> std::vector<P<T>> naive_twiddles(int k) {
  size_t N = size_t(1) << k, half = std::max<size_t>(N / 2, 1);
  std::vector<P<T>> R(static_cast<size_t>(std::max(k, 2)) + 1);
  R[0] = P<T>{1, 0}; R[1] = P<T>{-1, 0}; R[2] = P<T>{0, 1};
  for (int s = 2; s < k; ++s) {
    T re = 1 + R[s].re, im = R[s].im;
    T mag = std::sqrt(re * re + im * im);
    R[s + 1] = P<T>{re / mag, im / mag};
  }
  std::vector<P<T>> Tw(half);
  Tw[0] = P<T>{1, 0};
  for (size_t j = 1; j < N / 2; ++j) {
    int t = 63 - __builtin_clzll(static_cast<unsigned long long>(j));
    P<T> u = Tw[j - (size_t(1) << t)], r = R[k - t];
    Tw[j] = P<T>{u.re * r.re - u.im * r.im, u.re * r.im + u.im * r.re};
  }
  return Tw;
}

template <class T>
int naive_mul(const uint8_t *a, size_t na, const uint8_t *b, size_t nb, int digit_bits,
              uint8_t *out) {
  if (!a || !b || !out || na == 0 || nb == 0 || (digit_bits != 8 && digit_bits != 4))
    return ST_INVALID;
  std::fesetround(FE_TONEAREST);
  std::vector<uint32_t> x = to_digits(a, na, digit_bits), y = to_digits(b, nb, digit_bits);
  size_t L = x.size() + y.size() - 1;
  int k = ceil_log2(L);
  size_t N = size_t(1) << k;
  std::vector<P<T>> u(N, P<T>{0, 0}), v(N, P<T>{0, 0});
  for (size_t i = 0; i < x.size(); ++i) u[i].re = static_cast<T>(x[i]);
  for (size_t i = 0; i < y.size(); ++i) v[i].re = static_cast<T>(y[i]);
  std::vector<P<T>> Tw = naive_twiddles<T>(k);
  std::vector<P<T>> U = naive_fft(k, u, Tw, k, false), V = naive_fft(k, v, Tw, k, false);
  for (size_t i = 0; i < N; ++i)
    U[i] = P<T>{U[i].re * V[i].re - U[i].im * V[i].im, U[i].re * V[i].im + U[i].im * V[i].re};
  std::vector<P<T>> Z = naive_fft(k, U, Tw, k, true);
  std::vector<int64_t> c(L);
  for (size_t i = 0; i < L; ++i) {
    double v2 = std::nearbyint(static_cast<double>(Z[i].re) / static_cast<double>(N));
    c[i] = v2 < 0 ? 0 : static_cast<int64_t>(v2);
  }
  carry(c, digit_bits, out, na + nb);
  return ST_OK;
}

template <class T> std::vector<C<T>> from4(const double *p, size_t n) {
  std::vector<C<T>> v(n);
  for (size_t i = 0; i < n; ++i)
    v[i] = C<T>{I<T>{static_cast<T>(p[4 * i]), static_cast<T>(p[4 * i + 1])},
                I<T>{static_cast<T>(p[4 * i + 2]), static_cast<T>(p[4 * i + 3])}};
  return v;
}
template <class T> void to4(const std::vector<C<T>> &v, double *p) {
  for (size_t i = 0; i < v.size(); ++i) {
    p[4 * i] = v[i].re.lo; p[4 * i + 1] = v[i].re.hi;
    p[4 * i + 2] = v[i].im.lo; p[4 * i + 3] = v[i].im.hi;
  }
}

}  // namespace

// ===========================================================================
// C entry points (loaded through ctypes by the tests).  Interval arrays are
// passed as n x 4 doubles {re_lo, re_hi, im_lo, im_hi}.

extern "C" {

void oracle_set_mutation(int m) { g_mutation = m; }

// Exact size bookkeeping: number of digits per operand, L and N.
size_t oracle_fft_size(size_t na, size_t nb, int digit_bits) {
  size_t s = digit_bits == 4 ? 2 : 1;
  return size_t(1) << ceil_log2(s * (na + nb) - 1);
}

// Whole method: status, the product (na + nb bytes, zero-filled on failure),
// the largest real-part radius and the half-integer count.
int oracle_mul_f64(const uint8_t *a, size_t na, const uint8_t *b, size_t nb, int digit_bits,
                   int certify_mode, uint8_t *out, double *max_radius, int64_t *half_int) {
  return mul_impl<double>(a, na, b, nb, digit_bits, certify_mode, out, max_radius, half_int);
}
// Same method in single precision intervals (for probing how far FP32 reaches).
int oracle_mul_f32(const uint8_t *a, size_t na, const uint8_t *b, size_t nb, int digit_bits,
                   int certify_mode, uint8_t *out, double *max_radius, int64_t *half_int) {
  return mul_impl<float>(a, na, b, nb, digit_bits, certify_mode, out, max_radius, half_int);
}
// Non-rigorous point FFT variant, round to nearest (no certification).
int oracle_mul_naive_f64(const uint8_t *a, size_t na, const uint8_t *b, size_t nb,
                         int digit_bits, uint8_t *out) {
  return naive_mul<double>(a, na, b, nb, digit_bits, out);
}
int oracle_mul_naive_f32(const uint8_t *a, size_t na, const uint8_t *b, size_t nb,
                         int digit_bits, uint8_t *out) {
  return naive_mul<float>(a, na, b, nb, digit_bits, out);
}

// Enclosures of all N convolution outputs (after the inverse FFT and 1/N).
size_t oracle_conv_enclosure_f64(const uint8_t *a, size_t na, const uint8_t *b, size_t nb,
                                 int digit_bits, double *out4) {
  std::vector<uint32_t> x = to_digits(a, na, digit_bits), y = to_digits(b, nb, digit_bits);
  int k = 0;
  std::vector<C<double>> Z = convolve<double>(x, y, &k);
  to4(Z, out4);
  return Z.size();
}

// Interval DFT of length 2^k (inverse != 0: inverse DFT including 1/N).
void oracle_dft_f64(int k, int inverse, const double *in4, double *out4) {
  std::vector<C<double>> x = from4<double>(in4, size_t(1) << k);
  to4(dft<double>(k, x, inverse != 0), out4);
}

// Twiddle table T[j] ~ omega_N^j for 0 <= j < N/2 (N = 2^k, at least 1 entry).
void oracle_twiddles_f64(int k, double *out4) { to4(twiddles<double>(k), out4); }
// Roots R[s] ~ omega_{2^s}, 0 <= s <= k.
void oracle_roots_f64(int k, double *out4) { to4(roots<double>(k), out4); }

// Single real-interval operation on [a0,a1] (and [b0,b1]):
// op 0 add, 1 sub, 2 mul, 3 div, 4 sqrt.  Returns 0, or -1 if undefined.
int oracle_iop_f64(int op, const double *a2, const double *b2, double *r2) {
  I<double> a{a2[0], a2[1]}, b{b2 ? b2[0] : 0, b2 ? b2[1] : 0}, r{0, 0};
  switch (op) {
    case 0: r = iadd(a, b); break;
    case 1: r = isub(a, b); break;
    case 2: r = imul(a, b); break;
    case 3: if (!idiv(a, b, &r)) return -1; break;
    case 4: if (!isqrt(a, &r)) return -1; break;
    default: return -1;
  }
  r2[0] = r.lo; r2[1] = r.hi;
  return 0;
}
int oracle_iop_f32(int op, const float *a2, const float *b2, float *r2) {
  I<float> a{a2[0], a2[1]}, b{b2 ? b2[0] : 0.f, b2 ? b2[1] : 0.f}, r{0, 0};
  switch (op) {
    case 0: r = iadd(a, b); break;
    case 1: r = isub(a, b); break;
    case 2: r = imul(a, b); break;
    case 3: if (!idiv(a, b, &r)) return -1; break;
    case 4: if (!isqrt(a, &r)) return -1; break;
    default: return -1;
  }
  r2[0] = r.lo; r2[1] = r.hi;
  return 0;
}

// Complex interval product.
void oracle_cmul_f64(const double *a4, const double *b4, double *r4) {
  std::vector<C<double>> a = from4<double>(a4, 1), b = from4<double>(b4, 1);
  to4(std::vector<C<double>>{cmul(a[0], b[0])}, r4);
}

// Certification of n enclosures of which the first L are coefficients.
int oracle_certify_f64(const double *enc4, size_t n, size_t L, int mode, int64_t *c,
                       double *max_radius, int64_t *half_int) {
  std::vector<C<double>> Z = from4<double>(enc4, n);
  std::vector<int64_t> cv;
  int st = certify(Z, L, mode, &cv, max_radius, half_int);
  for (size_t i = 0; i < L; ++i) c[i] = cv[i];
  return st;
}

// Carry propagation of L non-negative coefficients in base 2^digit_bits into
// nout bytes.
void oracle_carry(const int64_t *c, size_t L, int digit_bits, uint8_t *out, size_t nout) {
  std::vector<int64_t> cv(c, c + L);
  carry(cv, digit_bits, out, nout);
}

}  // extern "C"
