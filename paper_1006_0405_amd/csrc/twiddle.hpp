// Certified twiddle-table generation (device kernels, host launcher).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace ssa {

// Writes tab[t] = (c_t, s_t), 0 <= t < 2^K, the doubles nearest the midpoints
// of rigorous enclosures of cos(2 pi t / 2^K) and sin(2 pi t / 2^K), and
// atomically maximises *ebits (bit pattern of a non-negative double, must be
// zero on entry) with an upper bound of every |component - stored value|.
// roots_scratch: device memory of twiddle_roots_bytes() bytes.  K <= 30.
hipError_t make_twiddles(int K, double2 *tab, unsigned long long *ebits, void *roots_scratch,
                         hipStream_t stream);
// Level tables: lv[2^l + u] = omega_{2^l}^u for 0 <= l <= K, 0 <= u < 2^l
// (2^(K+1) entries; lv[0] unused), so that the roots of one order are
// contiguous and a transform's twiddles occupy few cache lines.  Expects the
// top level lv[2^K ..] already written by make_twiddles; the lower levels are
// copies of its entries (u << (K - l)), so the bound e holds for all of them.
hipError_t make_level_tables(int K, double2 *lv, hipStream_t stream);
size_t twiddle_roots_bytes();

}  // namespace ssa
