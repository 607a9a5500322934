"""Seeded synthetic operands (shared by the tests, the benchmark and the smoke
check; it holds none of the multiplication's arithmetic).

The paper measures on uniformly random n-digit base-256 integers (section 3).
Each operand here is drawn with numpy's PCG64 generator: n uniform bytes, then
the top byte is redrawn from 1..255 so the number has exactly n digits.  Within
an instance `a` is drawn before `b`.
"""
import numpy as np

BATCH_COUNT = 4096
BATCH_MIN = 64
BATCH_MAX = 16384


def operand(rng, n):
    """n uniform random bytes, little-endian, top byte non-zero."""
    x = rng.integers(0, 256, n, dtype=np.uint8)
    if n > 0:
        x[n - 1] = rng.integers(1, 256)
    return x


def pair(seed, na, nb=None):
    """One product's operands (a first, then b) from one seed."""
    rng = np.random.default_rng(seed)
    a = operand(rng, na)
    b = operand(rng, na if nb is None else nb)
    return a, b


def all_ff(n):
    """The all-0xFF operand: worst-case coefficient growth."""
    return np.full(n, 0xFF, dtype=np.uint8)


def batch_lengths(seed=3, count=BATCH_COUNT, lo=BATCH_MIN, hi=BATCH_MAX):
    """Log-uniform operand lengths in [lo, hi]: floor(lo * (hi/lo)^u), u ~ U[0,1)."""
    rng = np.random.default_rng(seed)
    u = rng.random((count, 2))
    n = np.floor(lo * (hi / lo) ** u).astype(np.int64)
    n = np.minimum(n, hi)
    return rng, n[:, 0], n[:, 1]


def batch(seed=3, count=BATCH_COUNT, lo=BATCH_MIN, hi=BATCH_MAX):
    """The batch workload: count products with log-uniform lengths; operands
    drawn instance by instance (a then b) from the same generator after the
    lengths."""
    rng, na, nb = batch_lengths(seed, count, lo, hi)
    A, B = [], []
    for i in range(count):
        A.append(operand(rng, int(na[i])))
        B.append(operand(rng, int(nb[i])))
    return A, B
