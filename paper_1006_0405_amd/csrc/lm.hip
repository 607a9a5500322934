// Long multiplication (paper section 2.1, LM box) on the GPU: the O(n m)
// method the paper times the Schoenhage-Strassen product against (section 3).
//
// The column sums s_i = sum_j x_j y_{i-j} are exact integer dot products; the
// carry loop of the LM box is the library's carry scan over them (the same
// one as for the certified coefficients).  Work split: a workgroup of 256
// threads takes 1024 consecutive columns (4 per thread) and one slice of the
// j range; slices of the same columns add their partial sums with 64-bit
// atomics into the zeroed coefficient array.  Per slice, chunks of 1024 digits
// of x and the matching window of y are staged in LDS; each thread keeps the
// four y values its columns need for the current j in registers and shifts
// the window by one digit per step (one LDS read per four multiply-adds).
// A chunk's sums stay below 1024 * 255^2 < 2^32, so they accumulate in 32 bits.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"

namespace ssa {

namespace {

constexpr int LM_THREADS = 256;
constexpr int LM_COLS = 4 * LM_THREADS;  // columns per workgroup
constexpr int LM_CHUNK = 1024;           // digits of x per staged chunk

// Zero the coefficients and the product's statistics and carry state.
__global__ void k_lm_clear(const task *tkp, uint32_t L) {
  const task tk = *tkp;
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < L) tk.c[i] = 0ull;
  if (blockIdx.x == 0) {
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
}

// grid = (column tiles, j slices); slice s covers j in [s * span, (s + 1) * span).
__global__ __launch_bounds__(LM_THREADS) void k_lm(const task *tkp, uint32_t span) {
  __shared__ uint32_t sx[LM_CHUNK];
  __shared__ uint8_t sy[LM_COLS + LM_CHUNK + 4];
  const task tk = *tkp;
  const int64_t na = tk.na, nb = tk.nb, L = tk.L;
  const int64_t i0 = static_cast<int64_t>(blockIdx.x) * LM_COLS;
  const int t = threadIdx.x;
  // x_j contributes to columns j .. j + nb - 1: the tile needs j in
  // [i0 - nb + 1, i0 + LM_COLS - 1], within this slice and within x
  int64_t jlo = static_cast<int64_t>(blockIdx.y) * span;
  int64_t jhi = jlo + span;  // exclusive
  jlo = jlo > i0 - nb + 1 ? jlo : i0 - nb + 1;
  jlo = jlo > 0 ? jlo : 0;
  jhi = jhi < i0 + LM_COLS ? jhi : i0 + LM_COLS;
  jhi = jhi < na ? jhi : na;
  if (jlo >= jhi) return;  // uniform over the workgroup
  const int64_t i = i0 + 4 * t;  // this thread's first column
  unsigned long long acc[4] = {0ull, 0ull, 0ull, 0ull};
  for (int64_t j0 = jlo; j0 < jhi; j0 += LM_CHUNK) {
    const int64_t jn = (jhi - j0) < LM_CHUNK ? (jhi - j0) : LM_CHUNK;
    // y window: y_{i - j} for columns [i0, i0 + LM_COLS) and j in [j0, j0 + jn),
    // plus one below for the last shift: indices ybase + w, w < LM_COLS + LM_CHUNK + 1
    const int64_t ybase = i0 - j0 - LM_CHUNK;
    __syncthreads();  // the previous chunk is consumed
    for (int q = t; q < LM_CHUNK; q += LM_THREADS) {
      const int64_t j = j0 + q;
      sx[q] = (q < jn && j < na) ? static_cast<uint32_t>(tk.a[j]) : 0u;
    }
    for (int q = t; q < LM_COLS + LM_CHUNK + 4; q += LM_THREADS) {
      const int64_t y = ybase + q;
      sy[q] = (y >= 0 && y < nb) ? tk.b[y] : 0;
    }
    __syncthreads();
    // column i + u at step jj needs y_{i + u - j0 - jj} = sy[i + u - j0 - jj - ybase]
    const int off = static_cast<int>(i - j0 - ybase);  // = 4 t + LM_CHUNK
    uint32_t w[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) w[u] = sy[off + u];
    uint32_t s[4] = {0u, 0u, 0u, 0u};
    for (int jj = 0; jj < jn; ++jj) {
      const uint32_t x = sx[jj];
#pragma unroll
      for (int u = 0; u < 4; ++u) s[u] += x * w[u];
      // next step: columns see y one index lower
      w[3] = w[2];
      w[2] = w[1];
      w[1] = w[0];
      w[0] = sy[off - jj - 1];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] += s[u];
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (i + u < L && acc[u] != 0ull) atomicAdd(tk.c + i + u, acc[u]);
}

}  // namespace

hipError_t launch_long_mul(const task *d_task, const task &h_task, hipStream_t s) {
  const uint32_t L = h_task.L;
  hipLaunchKernelGGL(k_lm_clear, dim3((L + 255) / 256), dim3(256), 0, s, d_task, L);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const uint32_t tiles = (L + LM_COLS - 1) / LM_COLS;
  // enough workgroups to fill the GPU: split the j range into slices of at
  // least one chunk
  const uint32_t na = h_task.na;
  uint32_t slices = (2048 + tiles - 1) / tiles;
  const uint32_t max_slices = (na + LM_CHUNK - 1) / LM_CHUNK;
  slices = slices < max_slices ? slices : max_slices;
  slices = slices < 65535u ? slices : 65535u;
  const uint32_t span = (na + slices - 1) / slices;
  hipLaunchKernelGGL(k_lm, dim3(tiles, slices), dim3(LM_THREADS), 0, s, d_task, span);
  return hipGetLastError();
}

}  // namespace ssa
