// Exact last resort: the convolution by a number-theoretic transform.
//
// When every interval run refuses a product (an enclosure holds several
// integers), the paper's section 1 says that more precision or a different
// algorithm is needed.  This is the different algorithm: the same fast
// convolution (section 2.3) over the finite field Z_p, p = 2^64 - 2^32 + 1,
// instead of C -- the idea of the second Schoenhage-Strassen algorithm, which
// works over a finite ring and so needs no approximation at all (the paper's
// introduction).  p - 1 = 2^32 (2^32 - 1), so Z_p has roots of unity of every
// order 2^k, k <= 32, and 2^64 = 2^32 - 1 (mod p) makes reduction a few
// additions.  Every convolution coefficient of two base-256 operands is below
// min(na, nb) * 255^2 < p, so its residue IS the coefficient: the transform,
// the pointwise product and the inverse are exact, and no certification is
// needed.
//
// Layout: a product of N = 2^K points uses four arrays of N residues (uint64,
// 32 N bytes: the transform array of an interval product) and the level table
// lv[2^l + u] = w_{2^l}^u, 0 <= u < 2^l, l <= K, of the roots of unity
// w_{2^l} of order 2^l.  Each transform is a sequence of Stockham passes of
// radix R in {2, 4, 8, 16} (natural order in and out); a pass gives each
// thread R elements at stride N / R, multiplies them by w_{R Ns}^{r k} (powers
// of the one table entry w_{R Ns}^k), runs a length-R transform in registers
// and writes them at stride Ns (the length of the transforms the previous
// passes completed).  The inverse transform is
// the forward one read backwards: x_n = N^-1 X'_{-n mod N}, X' the forward
// transform of X.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"

namespace ssa {

namespace {

constexpr uint64_t P = 0xFFFFFFFF00000001ull;
constexpr uint64_t EPS = 0xFFFFFFFFull;  // 2^64 mod p

__device__ __forceinline__ uint64_t mp_add(uint64_t a, uint64_t b) {
  uint64_t s = a + b;
  // a + b < 2p: with a carry out of 2^64 the residue is s + 2^64 - p =
  // s + EPS (< p, no overflow); otherwise s, less p if s >= p
  if (s < a) return s + EPS;
  return s >= P ? s - P : s;
}

__device__ __forceinline__ uint64_t mp_sub(uint64_t a, uint64_t b) {
  // a - b + p when a < b: the wrapped difference a - b + 2^64, less EPS
  const uint64_t d = a - b;
  return a < b ? d - EPS : d;
}

// a b mod p for a, b < p: the 128-bit product hi 2^64 + lo with
// hi = h1 2^32 + h0, and 2^64 = 2^32 - 1, 2^96 = -1 (mod p):
// a b = lo - h1 + h0 (2^32 - 1)  (mod p).
__device__ __forceinline__ uint64_t mp_mul(uint64_t a, uint64_t b) {
  const uint64_t lo = a * b;
  const uint64_t hi = __umul64hi(a, b);
  const uint64_t h1 = hi >> 32, h0 = hi & EPS;
  uint64_t t = lo - h1;
  if (lo < h1) t -= EPS;           // borrow: + p
  const uint64_t u = (h0 << 32) - h0;  // h0 (2^32 - 1) < 2^64
  uint64_t s = t + u;
  if (s < t) s += EPS;             // carry: + 2^64 = + EPS (no overflow)
  return s >= P ? s - P : s;
}

__device__ __forceinline__ uint64_t mp_pow(uint64_t w, uint64_t e) {
  uint64_t r = 1;
  while (e) {
    if (e & 1) r = mp_mul(r, w);
    w = mp_mul(w, w);
    e >>= 1;
  }
  return r;
}

// lv[i] for 1 <= i < 2^(K+1): level l = floor(log2 i), entry u = i - 2^l,
// w_{2^l}^u with w_{2^l} = wK^(2^(K - l)).
__global__ void k_ntt_levels(int K, uint64_t wK, uint64_t *lv) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0 || i >= (2u << K)) return;
  const int l = 31 - __builtin_clz(i);
  const uint32_t u = i - (1u << l);
  uint64_t w = wK;
  for (int s = l; s < K; ++s) w = mp_mul(w, w);
  lv[i] = mp_pow(w, u);
}

// Length-R transform in registers, X_k = sum_r v_r w_R^{r k}, by recursive
// radix-2 decimation in time: X_k = E_k + w_R^k O_k, X_{k+R/2} = E_k - w_R^k O_k
// with E, O the length-R/2 transforms of the even and odd entries.  w holds
// the roots of the outermost length Rt, w[q] = w_Rt^q (q < Rt/2); at length R
// the root w_R^k is w[k WS], WS = Rt / R.
template <int R, int WS>
__device__ __forceinline__ void dft_r(uint64_t *v, const uint64_t *w) {
  if constexpr (R > 1) {
    uint64_t e[R / 2], o[R / 2];
#pragma unroll
    for (int r = 0; r < R / 2; ++r) {
      e[r] = v[2 * r];
      o[r] = v[2 * r + 1];
    }
    dft_r<R / 2, 2 * WS>(e, w);
    dft_r<R / 2, 2 * WS>(o, w);
#pragma unroll
    for (int k = 0; k < R / 2; ++k) {
      const uint64_t t = k == 0 ? o[k] : mp_mul(o[k], w[k * WS]);
      v[k] = mp_add(e[k], t);
      v[k + R / 2] = mp_sub(e[k], t);
    }
  }
}

// Source, sink and product of one pass.
enum { SRC_ARRAY = 0, SRC_DIGITS = 1 };
enum { DST_ARRAY = 0, DST_TIMES = 1, DST_COEFFS = 2 };

struct ntt_pass_args {
  const uint64_t *in;   // SRC_ARRAY
  const uint8_t *dig;   // SRC_DIGITS: operand bytes
  uint32_t nd;          // SRC_DIGITS: operand length
  uint64_t *out;        // DST_ARRAY / DST_TIMES: N residues; DST_COEFFS: coefficients
  const uint64_t *mul;  // DST_TIMES: out = transform * mul (elementwise)
  uint64_t ninv;        // DST_COEFFS: N^-1 mod p
};

// The product's statistics and carry state, reset by its first pass (block 0).
__device__ __forceinline__ void reset_product(const task &tk) {
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

// Input idx of a pass (SRC) and its output at position pos (DST).
template <int SRC>
__device__ __forceinline__ uint64_t ntt_get(const ntt_pass_args &p, uint32_t idx) {
  if constexpr (SRC == SRC_DIGITS)
    return idx < p.nd ? static_cast<uint64_t>(p.dig[idx]) : 0ull;
  else
    return p.in[idx];
}
template <int DST>
__device__ __forceinline__ void ntt_put(const ntt_pass_args &p, uint32_t N, uint32_t pos, uint64_t v) {
  if constexpr (DST == DST_ARRAY) {
    p.out[pos] = v;
  } else if constexpr (DST == DST_TIMES) {
    p.out[pos] = mp_mul(v, p.mul[pos]);
  } else {
    // inverse: x_n = N^-1 X'_{-n}; the residue is the coefficient itself
    p.out[(N - pos) & (N - 1)] = mp_mul(v, p.ninv);
  }
}

// One Stockham pass of radix R: thread j (< N/R) reads v_r = x[j + r N/R],
// k = j mod Ns, multiplies by w_{R Ns}^{r k}, transforms, and writes
// y[(j - k) R + k + r Ns].
template <int R, int SRC, int DST>
__global__ __launch_bounds__(256) void k_ntt_pass(ntt_pass_args p, int log_n, int log_ns,
                                                  const uint64_t *lv, const task *tk_reset) {
  if (tk_reset != nullptr && blockIdx.x == 0) reset_product(*tk_reset);  // the first pass
  const uint32_t N = 1u << log_n;
  const uint32_t M = N / R;  // threads of the pass
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  const uint32_t Ns = 1u << log_ns;
  const uint32_t k = j & (Ns - 1);
  uint64_t v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = ntt_get<SRC>(p, j + r * M);
  if (Ns > 1) {
    // w_{R Ns}^{r k} as powers of one entry of level R Ns: one load per thread,
    // contiguous over the lanes (strided reads of w^{r k} for every r would
    // touch up to R times the cache lines of the whole level)
    const uint64_t w1 = lv[(static_cast<size_t>(R) << log_ns) + k];
    uint64_t wr = w1;
    v[1] = mp_mul(v[1], w1);
#pragma unroll
    for (int r = 2; r < R; ++r) {
      wr = mp_mul(wr, w1);
      v[r] = mp_mul(v[r], wr);
    }
  }
  uint64_t w[R / 2];
#pragma unroll
  for (int q = 0; q < R / 2; ++q) w[q] = lv[R + q];  // w_R^q
  dft_r<R, 1>(v, w);
  const uint32_t base = (j - k) * R + k;
#pragma unroll
  for (int r = 0; r < R; ++r) ntt_put<DST>(p, N, base + r * Ns, v[r]);
}

// Fused pass of radix R = Q^2 (Q = 8 or 16): two radix-Q stages of the same
// Stockham step through LDS, so a transform takes about half the passes over
// HBM.  With r = r1 + Q r2 and q = q2 + Q q1 the length-R transform is
//   X_{q2 + Q q1} = sum_{r1} w_Q^{r1 q1} w_R^{r1 q2} sum_{r2} v_{r1 + Q r2} w_Q^{r2 q2}.
// A workgroup of 256 threads takes C = 256/Q consecutive values of j; thread
// (jl, a) first holds v_{a + Q r2} (r2 < Q), applies the pass twiddle
// w_{R Ns}^{(a + Q r2) k} (powers of the one entry w_{R Ns}^k), transforms over
// r2 and applies w_R^{a q2}; after the exchange it holds the values of its
// q2 = a for every r1, transforms over r1 and writes X_{a + Q q1} to
// y[(j - k) R + k + (a + Q q1) Ns].  QFAST (the first pass, Ns = 1: each j's
// outputs are contiguous) puts a in the fastest lanes so the writes coalesce;
// otherwise jl is fastest (loads and writes contiguous over j).
template <int Q, int SRC, int DST, bool QFAST>
__global__ __launch_bounds__(256) void k_ntt_pass2(ntt_pass_args p, int log_n, int log_ns,
                                                   const uint64_t *lv, const task *tk_reset) {
  constexpr int R = Q * Q;
  constexpr int C = 256 / Q;
  constexpr int JS = R + 1;  // LDS words per j (one spare word against bank conflicts)
  __shared__ uint64_t sh[C * JS];
  if (tk_reset != nullptr && blockIdx.x == 0) reset_product(*tk_reset);
  const uint32_t N = 1u << log_n;
  const uint32_t M = N / R;
  const uint32_t Ns = 1u << log_ns;
  const int t = threadIdx.x;
  const int jl = QFAST ? t / Q : t % C;
  const int a = QFAST ? t % Q : t / C;
  const uint32_t j = blockIdx.x * C + jl;  // grid = M / C: every j exists
  const uint32_t k = j & (Ns - 1);
  uint64_t v[Q];
#pragma unroll
  for (int r2 = 0; r2 < Q; ++r2) v[r2] = ntt_get<SRC>(p, j + static_cast<uint32_t>(a + Q * r2) * M);
  if (Ns > 1) {
    const uint64_t W = lv[(static_cast<size_t>(R) << log_ns) + k];  // w_{R Ns}^k
    uint64_t f = 1, WQ = W;
    for (int b = a, wb = 0; b; b >>= 1, ++wb) {  // f = W^a, a < Q
      uint64_t x = W;
      for (int s2 = 0; s2 < wb; ++s2) x = mp_mul(x, x);
      if (b & 1) f = mp_mul(f, x);
    }
#pragma unroll
    for (int s2 = 1; s2 < Q; s2 <<= 1) WQ = mp_mul(WQ, WQ);  // W^Q
#pragma unroll
    for (int r2 = 0; r2 < Q; ++r2) {
      if (r2 > 0) f = mp_mul(f, WQ);
      v[r2] = mp_mul(v[r2], f);
    }
  }
  uint64_t wq[Q / 2];
#pragma unroll
  for (int q = 0; q < Q / 2; ++q) wq[q] = lv[Q + q];  // w_Q^q
  dft_r<Q, 1>(v, wq);
  if (a > 0) {
#pragma unroll
    for (int q2 = 1; q2 < Q; ++q2) v[q2] = mp_mul(v[q2], lv[R + a * q2]);  // w_R^{a q2}
  }
#pragma unroll
  for (int q2 = 0; q2 < Q; ++q2) sh[jl * JS + q2 * Q + a] = v[q2];
  __syncthreads();
#pragma unroll
  for (int r1 = 0; r1 < Q; ++r1) v[r1] = sh[jl * JS + a * Q + r1];
  dft_r<Q, 1>(v, wq);
  const uint32_t base = (j - k) * R + k;
#pragma unroll
  for (int q1 = 0; q1 < Q; ++q1) ntt_put<DST>(p, N, base + static_cast<uint32_t>(a + Q * q1) * Ns, v[q1]);
}

template <int SRC, int DST, bool QFAST>
hipError_t launch_pass2(int Q, const ntt_pass_args &a, int log_n, int log_ns, const uint64_t *lv,
                        const task *tk_reset, hipStream_t s) {
  const uint32_t R = static_cast<uint32_t>(Q) * Q, C = 256u / Q;
  const dim3 grid(((1u << log_n) / R) / C);
  if (Q == 16)
    hipLaunchKernelGGL((k_ntt_pass2<16, SRC, DST, QFAST>), grid, dim3(256), 0, s, a, log_n, log_ns,
                       lv, tk_reset);
  else
    hipLaunchKernelGGL((k_ntt_pass2<8, SRC, DST, QFAST>), grid, dim3(256), 0, s, a, log_n, log_ns,
                       lv, tk_reset);
  return hipGetLastError();
}

template <int SRC, int DST>
hipError_t launch_pass_r(int R, const ntt_pass_args &a, int log_n, int log_ns, const uint64_t *lv,
                         const task *tk_reset, hipStream_t s) {
  const uint32_t threads = (1u << log_n) / R;
  const dim3 grid((threads + 255) / 256);
  switch (R) {
    case 2:
      hipLaunchKernelGGL((k_ntt_pass<2, SRC, DST>), grid, dim3(256), 0, s, a, log_n, log_ns, lv, tk_reset);
      break;
    case 4:
      hipLaunchKernelGGL((k_ntt_pass<4, SRC, DST>), grid, dim3(256), 0, s, a, log_n, log_ns, lv, tk_reset);
      break;
    case 8:
      hipLaunchKernelGGL((k_ntt_pass<8, SRC, DST>), grid, dim3(256), 0, s, a, log_n, log_ns, lv, tk_reset);
      break;
    default:
      hipLaunchKernelGGL((k_ntt_pass<16, SRC, DST>), grid, dim3(256), 0, s, a, log_n, log_ns, lv, tk_reset);
      break;
  }
  return hipGetLastError();
}

// Next pass of a length-2^log_n transform after `done` levels: a fused pass
// of radix 256 while eight or more levels remain (2^12 points and more: a
// workgroup takes 16 values of j), then of radix 64 while six remain (2^11
// points and more), then single passes of radix 16, and what is left.
// Returns log2 of the radix; *Q is the fused pass's Q (0: a single pass).
int next_pass(int log_n, int done, int *Q) {
  const int rem = log_n - done;
  *Q = 0;
  if (rem >= 8 && log_n >= 12) {
    *Q = 16;
    return 8;
  }
  if (rem >= 6 && log_n >= 11) {
    *Q = 8;
    return 6;
  }
  return rem >= 4 ? 4 : rem;
}

}  // namespace

hipError_t make_ntt_levels(int K, uint64_t wK, uint64_t *lv, hipStream_t s) {
  const uint32_t n = 2u << K;
  hipLaunchKernelGGL(k_ntt_levels, dim3((n + 255) / 256), dim3(256), 0, s, K, wK, lv);
  return hipGetLastError();
}

// One transform of length 2^log_n through the two buffers b0, b1, starting
// from the digits (dig, nd) or from the array `in` (which may be b0 or b1);
// with `mul`, the last pass writes the elementwise product with mul; with
// `coeffs`, the last pass writes the inverse transform's coefficients there.
// Returns the buffer holding the result (unused with coeffs).
static hipError_t transform(const uint8_t *dig, uint32_t nd, const uint64_t *in, int log_n,
                            const uint64_t *lv, uint64_t *b0, uint64_t *b1, const uint64_t *mul,
                            uint64_t *coeffs, uint64_t ninv, const task *tk_reset, hipStream_t s,
                            const uint64_t **result) {
  int done = 0;
  const uint64_t *src = in;
  uint64_t *dst = (in == b0) ? b1 : b0;
  while (done < log_n) {
    int Q = 0;
    const int lr = next_pass(log_n, done, &Q);
    const int R = 1 << lr;
    const bool first = done == 0, last = done + lr == log_n;
    ntt_pass_args a{};
    a.in = src;
    a.dig = dig;
    a.nd = nd;
    a.out = dst;
    a.mul = mul;
    a.ninv = ninv;
    const task *rs = first ? tk_reset : nullptr;
    hipError_t e;
    if (Q != 0) {  // fused (never both the first and the last pass: log_n >= 11)
      if (first && dig != nullptr) e = launch_pass2<SRC_DIGITS, DST_ARRAY, true>(Q, a, log_n, done, lv, rs, s);
      else if (first) e = launch_pass2<SRC_ARRAY, DST_ARRAY, true>(Q, a, log_n, done, lv, rs, s);
      else if (last && coeffs) {
        a.out = coeffs;
        e = launch_pass2<SRC_ARRAY, DST_COEFFS, false>(Q, a, log_n, done, lv, rs, s);
      } else if (last && mul) {
        e = launch_pass2<SRC_ARRAY, DST_TIMES, false>(Q, a, log_n, done, lv, rs, s);
      } else {
        e = launch_pass2<SRC_ARRAY, DST_ARRAY, false>(Q, a, log_n, done, lv, rs, s);
      }
    } else if (first && dig != nullptr) {
      if (last && mul) e = launch_pass_r<SRC_DIGITS, DST_TIMES>(R, a, log_n, done, lv, rs, s);
      else e = launch_pass_r<SRC_DIGITS, DST_ARRAY>(R, a, log_n, done, lv, rs, s);
    } else if (last && coeffs) {
      a.out = coeffs;
      e = launch_pass_r<SRC_ARRAY, DST_COEFFS>(R, a, log_n, done, lv, rs, s);
    } else if (last && mul) {
      e = launch_pass_r<SRC_ARRAY, DST_TIMES>(R, a, log_n, done, lv, rs, s);
    } else {
      e = launch_pass_r<SRC_ARRAY, DST_ARRAY>(R, a, log_n, done, lv, rs, s);
    }
    if (e != hipSuccess) return e;
    done += lr;
    src = dst;
    dst = (dst == b0) ? b1 : b0;
  }
  *result = src;
  return hipSuccess;
}

hipError_t launch_ntt_product(const task *d_task, const task &h_task, int log_n, const uint64_t *lv,
                              uint64_t ninv, hipStream_t s) {
  uint64_t *buf = reinterpret_cast<uint64_t *>(h_task.ya);
  const size_t N = size_t(1) << log_n;
  uint64_t *b0 = buf, *b1 = buf + N, *b2 = buf + 2 * N, *b3 = buf + 3 * N;
  const uint64_t *A = nullptr, *C = nullptr, *unused = nullptr;
  // forward transform of a (its first pass resets the product's statistics
  // and carry state), then b's, whose last pass multiplies by A's
  hipError_t e = transform(h_task.a, h_task.na, nullptr, log_n, lv, b0, b1, nullptr, nullptr, 0,
                           d_task, s, &A);
  if (e == hipSuccess)
    e = transform(h_task.b, h_task.nb, nullptr, log_n, lv, b2, b3, A, nullptr, 0, nullptr, s, &C);
  // the inverse, read backwards and scaled, into the coefficients
  if (e == hipSuccess)
    e = transform(nullptr, 0, C, log_n, lv, b2, b3, nullptr, reinterpret_cast<uint64_t *>(h_task.c),
                  ninv, nullptr, s, &unused);
  return e;
}

}  // namespace ssa
