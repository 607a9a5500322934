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
size_t twiddle_roots_bytes();

}  // namespace ssa
