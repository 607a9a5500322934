"""Exact references that pin the oracle (and, through it, the GPU library).

None of these uses the FFT or interval arithmetic: they are the schoolbook
long multiplication of section 2.1, CPython's exact integer product, the closed
form of (B^n - 1)(B^m - 1), and exact integer convolution.
"""
import numpy as np


def to_int(x):
    return int.from_bytes(np.asarray(x, dtype=np.uint8).tobytes(), "little")


def int_product(a, b):
    """CPython integer product as len(a)+len(b) little-endian bytes."""
    return np.frombuffer((to_int(a) * to_int(b)).to_bytes(len(a) + len(b), "little"),
                         dtype=np.uint8)


def long_multiplication(x, y, base=256):
    """The long multiplication box of section 2.1, digit by digit: for every
    output position i the column sum s over j, then z_i = (s + c) mod b and
    c = floor((s + c) / b).  The inner column sum is a dot product of the
    digit slices (same sum, evaluated by numpy in exact int64)."""
    x = np.asarray(x, dtype=np.int64)
    y = np.asarray(y, dtype=np.int64)
    n, m = len(x), len(y)
    z = np.zeros(n + m, dtype=np.int64)
    c = 0
    for i in range(n + m):
        j0, j1 = max(0, i - m + 1), min(n - 1, i)
        s = 0
        if j0 <= j1:
            # y_{i-j} for j = j0..j1 is y[i-j1 .. i-j0] reversed
            s = int(np.dot(x[j0:j1 + 1], y[i - j1:i - j0 + 1][::-1]))
        z[i] = (s + c) % base
        c = (s + c) // base
    assert c == 0
    return z.astype(np.uint8)


def all_ff_product(n, m):
    """Bytes of (256^n - 1)(256^m - 1) = 256^(n+m) - 256^n - 256^m + 1, n >= m:
    z_0 = 1, z_1..z_{m-1} = 0, z_m..z_{n-1} = 0xFF, z_n = 0xFE,
    z_{n+1}..z_{n+m-1} = 0xFF (for n == m the run z_m..z_{n-1} is empty)."""
    if n < m:
        n, m = m, n
    z = np.zeros(n + m, dtype=np.uint8)
    z[0] = 1
    z[m:n] = 0xFF
    z[n] = 0xFE
    z[n + 1:] = 0xFF
    return z


def exact_convolution(x, y):
    """c_i = sum_j x_j y_{i-j} in exact integers."""
    x = np.asarray(x, dtype=np.int64)
    y = np.asarray(y, dtype=np.int64)
    # int64 is exact here: every column sum is at most min(n, m) * 255^2.
    if len(x) * len(y) <= 10_000_000_000:
        return np.convolve(x, y)
    raise ValueError("too large for a direct convolution; sample columns instead")


def all_ff_coefficients(na, nb, base=256):
    """(b-1)^2 * number of terms in column i: min(i, na-1) - max(0, i-nb+1) + 1."""
    L = na + nb - 1
    i = np.arange(L, dtype=np.int64)
    cnt = np.minimum(i, na - 1) - np.maximum(0, i - nb + 1) + 1
    return (base - 1) ** 2 * cnt


def nibbles(x):
    """Base-16 digits of a byte vector, low nibble first."""
    x = np.asarray(x, dtype=np.uint8)
    d = np.empty(2 * len(x), dtype=np.uint8)
    d[0::2] = x & 15
    d[1::2] = x >> 4
    return d
