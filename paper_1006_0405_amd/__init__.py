"""Rigorous complex-interval Schoenhage-Strassen integer multiplication on
MI355X (gfx950).

The multiplication runs in the HIP kernels of libssa.so behind the C ABI in
include/ssa.h; `binding` is its thin ctypes binding.  `workloads` holds the
seeded synthetic operands used by the tests and the benchmark.
"""
__all__ = ["binding", "workloads"]
