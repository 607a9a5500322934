"""Pins of the CPU oracle against what the paper and mathematics fix.

The oracle is the reference the GPU library is checked against, so it is
itself checked here against references that share none of its arithmetic:

* schoolbook long multiplication (paper section 2.1, long multiplication box);
* the CPython integer product;
* the closed form of (256^n - 1)(256^m - 1) (worst-case coefficient growth);
* hand-worked tiny products (tests/golden/tiny_products.txt);
* exact integer convolution coefficients inside every enclosure;
* DFT special cases from the Lemma of section 2.2 and the DFT definition
  evaluated in 200-bit mpmath interval arithmetic;
* twiddle enclosures against mpmath interval cos/sin;
* directed-rounding primitives against exact rational arithmetic;
* certification cases (section 1: unique integer, else an error).

Enclosure radii and the certification frontier are "parity unpinned": the paper
prints no values for them (its timing figure is missing).
"""
import os
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import oracle
from paper_1006_0405_amd.workloads import all_ff, pair
from pins import (all_ff_coefficients, all_ff_product, exact_convolution, int_product,
                  long_multiplication, nibbles)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def read_tiny_products():
    rows = []
    for line in open(os.path.join(GOLDEN, "tiny_products.txt")):
        if line.startswith("#") or not line.strip():
            continue
        a, b, c, z = [p.split() for p in line.split("|")]
        rows.append((np.array([int(x, 16) for x in a], np.uint8),
                     np.array([int(x, 16) for x in b], np.uint8),
                     [int(x) for x in c],
                     np.array([int(x, 16) for x in z], np.uint8)))
    return rows


# ---------------------------------------------------------------------------
# Products


@pytest.mark.parametrize("row", read_tiny_products(), ids=lambda r: "x".join(
    "".join("%02x" % v for v in r[i]) for i in (0, 1)))
def test_tiny_products_golden(row):
    a, b, c, z = row
    st, out, rad, _ = oracle.mul(a, b)
    assert st == oracle.ST_OK
    assert out.tolist() == z.tolist()
    enc = oracle.conv_enclosure(a, b)
    for i, ci in enumerate(c):
        assert enc[i, 0] <= ci <= enc[i, 1]


@pytest.mark.parametrize("na,nb,seed", [(1, 1, 0), (1, 9, 1), (9, 1, 2), (2, 3, 3), (17, 33, 4),
                                        (64, 64, 5), (100, 37, 6), (255, 256, 7), (1000, 24, 8),
                                        (1024, 1024, 9), (2047, 1500, 10)])
def test_against_long_multiplication(na, nb, seed):
    a, b = pair(seed, na, nb)
    ref = long_multiplication(a, b)
    st, out, _, _ = oracle.mul(a, b)
    assert st == oracle.ST_OK
    assert np.array_equal(out, ref)


@pytest.mark.parametrize("n,m", [(1, 1), (2, 1), (5, 5), (4, 2), (2, 4), (100, 3), (1024, 1024),
                                 (3000, 2999)])
def test_all_ff_closed_form(n, m):
    a, b = all_ff(n), all_ff(m)
    st, out, _, _ = oracle.mul(a, b)
    assert st == oracle.ST_OK
    assert np.array_equal(out, all_ff_product(n, m))
    assert np.array_equal(out, long_multiplication(a, b))


def test_config1_product():
    a, b = pair(1, 1024)
    st, out, rad, _ = oracle.mul(a, b)
    assert st == oracle.ST_OK
    assert np.array_equal(out, int_product(a, b))
    assert np.array_equal(out, long_multiplication(a, b))
    assert 0 < rad < 0.5


def test_leading_zeros_and_zero_operands():
    rng = np.random.default_rng(11)
    a = rng.integers(0, 256, 50, dtype=np.uint8)
    a[-10:] = 0
    b = np.zeros(30, np.uint8)
    for x, y in [(a, b), (b, a), (a, a), (b, b)]:
        st, out, _, _ = oracle.mul(x, y)
        assert st == oracle.ST_OK
        assert np.array_equal(out, int_product(x, y))


@pytest.mark.parametrize("na,nb,seed", [(1, 1, 0), (3, 2, 1), (64, 64, 2), (500, 300, 3),
                                        (1024, 1024, 4)])
def test_base16_split(na, nb, seed):
    a, b = pair(seed, na, nb)
    st, out, rad, _ = oracle.mul(a, b, digit_bits=4)
    assert st == oracle.ST_OK
    assert np.array_equal(out, int_product(a, b))
    # the base-16 convolution enclosures contain the exact nibble convolution
    enc = oracle.conv_enclosure(a, b, digit_bits=4)
    c = exact_convolution(nibbles(a), nibbles(b))
    assert np.all(enc[:len(c), 0] <= c) and np.all(c <= enc[:len(c), 1])


def test_invalid_arguments():
    a = np.zeros(0, np.uint8)
    st, _, _, _ = oracle.mul(a, np.ones(3, np.uint8))
    assert st == oracle.ST_INVALID
    st, _, _, _ = oracle.mul(np.ones(3, np.uint8), np.ones(3, np.uint8), digit_bits=5)
    assert st == oracle.ST_INVALID


# ---------------------------------------------------------------------------
# Enclosures contain the exact coefficients


@pytest.mark.parametrize("na,nb,seed", [(1, 1, 0), (7, 5, 1), (300, 200, 2), (1024, 1024, 3)])
def test_enclosures_contain_exact_convolution(na, nb, seed):
    a, b = pair(seed, na, nb)
    enc = oracle.conv_enclosure(a, b)
    c = exact_convolution(a, b)
    L = len(c)
    assert enc.shape[0] == oracle.fft_size(na, nb)
    assert np.all(enc[:, 0] <= enc[:, 1]) and np.all(enc[:, 2] <= enc[:, 3])
    assert np.all(enc[:L, 0] <= c) and np.all(c <= enc[:L, 1])
    assert np.all(enc[:, 2] <= 0) and np.all(enc[:, 3] >= 0)
    assert np.all(enc[L:, 0] <= 0) and np.all(enc[L:, 1] >= 0)


def test_enclosures_contain_all_ff_coefficients():
    na, nb = 2000, 1300
    enc = oracle.conv_enclosure(all_ff(na), all_ff(nb))
    c = all_ff_coefficients(na, nb)
    assert np.all(enc[:len(c), 0] <= c) and np.all(c <= enc[:len(c), 1])


# ---------------------------------------------------------------------------
# DFT (section 2.2)


def _thin(vals):
    v = np.asarray(vals, dtype=np.complex128)
    x = np.zeros((len(v), 4))
    x[:, 0] = x[:, 1] = v.real
    x[:, 2] = x[:, 3] = v.imag
    return x


@pytest.mark.parametrize("k", [0, 1, 2, 3, 6, 10])
def test_dft_of_unit_impulse_is_all_ones_exactly(k):
    N = 1 << k
    e0 = np.zeros(N)
    e0[0] = 1
    X = oracle.dft(k, _thin(e0))
    assert np.all(X[:, 0] == 1) and np.all(X[:, 1] == 1)
    assert np.all(X[:, 2] == 0) and np.all(X[:, 3] == 0)


@pytest.mark.parametrize("k", [1, 2, 5, 9])
def test_dft_of_ones_is_n_times_impulse(k):
    # Lemma of section 2.2: sum_i omega^{ik} = 0 for 0 < k < n.
    N = 1 << k
    X = oracle.dft(k, _thin(np.ones(N)))
    assert X[0, 0] <= N <= X[0, 1]
    assert np.all(X[1:, 0] <= 0) and np.all(X[1:, 1] >= 0)
    assert np.all(X[:, 2] <= 0) and np.all(X[:, 3] >= 0)


def _mp_contains(lo, hi, ivx):
    return mpmath.mpf(lo) <= ivx.a and ivx.b <= mpmath.mpf(hi)


def _omega_iv(m, N):
    """200-bit interval enclosure of (cos, sin)(2 pi m / N); exact at multiples
    of a quarter turn."""
    m %= N
    if (4 * m) % N == 0:
        q = 4 * m // N
        return [(mpmath.iv.mpf(c), mpmath.iv.mpf(s)) for c, s in [(1, 0), (0, 1), (-1, 0), (0, -1)]][q]
    ang = 2 * mpmath.iv.pi * m / N
    return mpmath.iv.cos(ang), mpmath.iv.sin(ang)


@pytest.mark.parametrize("k", [2, 3, 4, 5])
def test_dft_matches_definition_in_high_precision(k):
    """x_hat_i = sum_j x_j omega^{ij}, omega = e^{+2 pi i / n}, evaluated in
    200-bit interval arithmetic, lies inside the oracle's enclosure."""
    N = 1 << k
    rng = np.random.default_rng(k)
    x = rng.integers(0, 256, N).astype(float)
    X = oracle.dft(k, _thin(x))
    mpmath.iv.prec = 200
    for i in range(N):
        re = mpmath.iv.mpf(0)
        im = mpmath.iv.mpf(0)
        for j in range(N):
            c, s = _omega_iv(i * j, N)
            re += int(x[j]) * c
            im += int(x[j]) * s
        assert _mp_contains(X[i, 0], X[i, 1], re), (i, X[i], re)
        assert _mp_contains(X[i, 2], X[i, 3], im), (i, X[i], im)


@pytest.mark.parametrize("k", [3, 8, 12])
def test_dft_of_e1_contains_powers_of_omega(k):
    N = 1 << k
    e1 = np.zeros(N)
    e1[1] = 1
    X = oracle.dft(k, _thin(e1))
    mpmath.iv.prec = 200
    for i in list(range(0, N, max(1, N // 64))) + [N // 4, N // 2, N - 1]:
        c, s = _omega_iv(i, N)
        assert _mp_contains(X[i, 0], X[i, 1], c)
        assert _mp_contains(X[i, 2], X[i, 3], s)


@pytest.mark.parametrize("k", [0, 1, 4, 11])
def test_dft_inverse_round_trip_contains_input(k):
    N = 1 << k
    rng = np.random.default_rng(100 + k)
    x = rng.integers(0, 256, N).astype(float)
    Y = oracle.dft(k, oracle.dft(k, _thin(x)), inverse=True)
    assert np.all(Y[:, 0] <= x) and np.all(x <= Y[:, 1])
    assert np.all(Y[:, 2] <= 0) and np.all(Y[:, 3] >= 0)
    assert np.max(Y[:, 1] - Y[:, 0]) < 1e-6


# ---------------------------------------------------------------------------
# Twiddles and roots (section 2.2 recurrence)


@pytest.mark.parametrize("k", [2, 3, 7, 12, 18])
def test_twiddles_contain_true_values(k):
    N = 1 << k
    T = oracle.twiddles(k)
    assert T.shape[0] == N // 2
    mpmath.iv.prec = 200
    idx = sorted(set(list(range(0, N // 2, max(1, N // 512))) + [1, N // 8, N // 4, N // 2 - 1]))
    for j in idx:
        if j >= N // 2:
            continue
        c, s = _omega_iv(j, N)
        assert _mp_contains(T[j, 0], T[j, 1], c), (k, j)
        assert _mp_contains(T[j, 2], T[j, 3], s), (k, j)
        # width: the rectangular products widen, but stay far below 1e-12
        assert T[j, 1] - T[j, 0] <= 1e-12 and T[j, 3] - T[j, 2] <= 1e-12
    # omega^{N/4} = i exactly
    assert tuple(T[N // 4]) == (0.0, 0.0, 1.0, 1.0)


def test_roots_special_values_and_containment():
    R = oracle.roots(20)
    assert tuple(R[0]) == (1, 1, 0, 0)
    assert tuple(R[1]) == (-1, -1, 0, 0)
    assert tuple(R[2]) == (0, 0, 1, 1)
    mpmath.iv.prec = 200
    for s in range(3, 21):
        ang = 2 * mpmath.iv.pi / (1 << s)
        assert _mp_contains(R[s, 0], R[s, 1], mpmath.iv.cos(ang))
        assert _mp_contains(R[s, 2], R[s, 3], mpmath.iv.sin(ang))


# ---------------------------------------------------------------------------
# Directed rounding primitives (section 2.5, outward rounding)


def _edge_doubles():
    v = [0.0, -0.0, 1.0, -1.0, 0.5, 3.0, 1e-310, -1e-310, 5e-324, 2.0 ** 52, 2.0 ** 53 - 1,
         2.0 ** 53 + 2, 1.0 + 2.0 ** -52, 1.0 - 2.0 ** -53, 0.1, -0.7, 1e300, 123456789.123]
    return v


def _random_doubles(rng, n):
    m = rng.standard_normal(n) * np.exp2(rng.integers(-60, 60, n))
    return list(m)


def _adjacent_below(x, exact):
    """x is the largest double <= exact."""
    return Fraction(x) <= exact and Fraction(np.nextafter(x, np.inf)) > exact


def _adjacent_above(x, exact):
    return Fraction(x) >= exact and Fraction(np.nextafter(x, -np.inf)) < exact


@pytest.mark.parametrize("op", ["add", "sub", "mul", "div"])
def test_directed_rounding_is_adjacent_f64(op):
    rng = np.random.default_rng(hash(op) % 1000)
    xs = _edge_doubles() + _random_doubles(rng, 300)
    ys = list(reversed(_edge_doubles())) + _random_doubles(rng, 300)
    for a, b in zip(xs, ys):
        if op == "div" and b == 0:
            assert oracle.iop(op, (a, a), (b, b)) is None
            continue
        fa, fb = Fraction(a), Fraction(b)
        exact = {"add": fa + fb, "sub": fa - fb, "mul": fa * fb, "div": fa / fb if b else None}[op]
        lo, hi = oracle.iop(op, (a, a), (b, b))
        if abs(exact) > Fraction(np.finfo(np.float64).max):
            continue
        assert _adjacent_below(lo, exact), (op, a, b, lo)
        assert _adjacent_above(hi, exact), (op, a, b, hi)


def test_directed_rounding_is_adjacent_f32():
    rng = np.random.default_rng(7)
    xs = (rng.standard_normal(300) * np.exp2(rng.integers(-20, 20, 300))).astype(np.float32)
    ys = (rng.standard_normal(300) * np.exp2(rng.integers(-20, 20, 300))).astype(np.float32)
    for op in ("add", "sub", "mul", "div"):
        for a, b in zip(xs, ys):
            fa, fb = Fraction(float(a)), Fraction(float(b))
            exact = {"add": fa + fb, "sub": fa - fb, "mul": fa * fb, "div": fa / fb}[op]
            lo, hi = oracle.iop(op, (a, a), (b, b), precision="f32")
            assert Fraction(float(lo)) <= exact < Fraction(float(np.nextafter(lo, np.float32(np.inf))))
            assert Fraction(float(hi)) >= exact > Fraction(float(np.nextafter(hi, np.float32(-np.inf))))


def test_directed_sqrt_is_adjacent():
    rng = np.random.default_rng(3)
    for x in [0.0, 1.0, 2.0, 3.0, 4.0, 0.5, 1e-300, 5e-324, 2.0 ** 52 + 1] + list(np.abs(_random_doubles(rng, 200))):
        lo, hi = oracle.iop("sqrt", (x, x))
        fx = Fraction(x)
        assert Fraction(lo) ** 2 <= fx and Fraction(hi) ** 2 >= fx
        if Fraction(lo) ** 2 != fx:
            assert Fraction(np.nextafter(lo, np.inf)) ** 2 > fx
            assert Fraction(np.nextafter(hi, -np.inf)) ** 2 < fx
        else:
            assert lo == hi
    assert oracle.iop("sqrt", (-1.0, 1.0)) is None


def test_interval_products_contain_all_point_products():
    rng = np.random.default_rng(5)
    for _ in range(300):
        a = np.sort(rng.standard_normal(2) * 10)
        b = np.sort(rng.standard_normal(2) * 10)
        lo, hi = oracle.iop("mul", a, b)
        for u in np.linspace(a[0], a[1], 5):
            for v in np.linspace(b[0], b[1], 5):
                assert Fraction(lo) <= Fraction(u) * Fraction(v) <= Fraction(hi)
        # sharp up to one rounding: the end-point extremes are attained
        ex = [Fraction(x) * Fraction(y) for x in a for y in b]
        assert _adjacent_below(lo, min(ex)) and _adjacent_above(hi, max(ex))
    assert oracle.iop("div", (1.0, 2.0), (-1.0, 1.0)) is None


def test_complex_interval_product_contains_point_products():
    rng = np.random.default_rng(6)
    for _ in range(100):
        z = np.concatenate([np.sort(rng.standard_normal(2)), np.sort(rng.standard_normal(2))])
        w = np.concatenate([np.sort(rng.standard_normal(2)), np.sort(rng.standard_normal(2))])
        r = oracle.cmul(z, w)
        for zr in z[:2]:
            for zi in z[2:]:
                for wr in w[:2]:
                    for wi in w[2:]:
                        pr = Fraction(zr) * Fraction(wr) - Fraction(zi) * Fraction(wi)
                        pi = Fraction(zr) * Fraction(wi) + Fraction(zi) * Fraction(wr)
                        assert Fraction(r[0]) <= pr <= Fraction(r[1])
                        assert Fraction(r[2]) <= pi <= Fraction(r[3])


# ---------------------------------------------------------------------------
# Certification (section 1) and carries (section 2.4)


CERTIFY_CASES = [
    ((2.6, 3.4), oracle.ST_OK, 3, 0),
    ((3.0, 3.0), oracle.ST_OK, 3, 0),
    ((-0.2, 0.3), oracle.ST_OK, 0, 0),
    ((3.0, 3.9), oracle.ST_OK, 3, 1),
    ((2.5, 3.5), oracle.ST_OK, 3, 1),
    ((2.9, 4.1), oracle.ST_TOO_WIDE, None, 1),
    ((3.2, 3.8), oracle.ST_INTERNAL, None, 1),
    ((-1.2, -0.9), oracle.ST_INTERNAL, None, 0),
    ((-1.3, 5.0), oracle.ST_TOO_WIDE, None, 1),
]


@pytest.mark.parametrize("case", CERTIFY_CASES, ids=lambda c: str(c[0]))
def test_certify_cases(case):
    (lo, hi), st_expect, value, half = case
    enc = np.array([[lo, hi, -1e-9, 1e-9]])
    st, c, rad, nhalf = oracle.certify(enc, 1)
    assert st == st_expect
    if value is not None:
        assert c[0] == value
    assert nhalf == half
    assert rad >= (hi - lo) / 2


def test_certify_strict_half_integer_mode():
    enc = np.array([[2.5, 3.5, 0, 0]])
    assert oracle.certify(enc, 1, mode=1)[0] == oracle.ST_TOO_WIDE
    assert oracle.certify(enc, 1, mode=0)[0] == oracle.ST_OK


def test_certify_imaginary_and_tail_invariants():
    enc = np.array([[3.0, 3.0, 0.1, 0.2]])
    assert oracle.certify(enc, 1)[0] == oracle.ST_INTERNAL
    enc = np.array([[3.0, 3.0, 0, 0], [0.5, 0.6, 0, 0]])
    assert oracle.certify(enc, 1)[0] == oracle.ST_INTERNAL
    enc = np.array([[3.0, 3.0, 0, 0], [-0.5, 0.6, 0, 0]])
    assert oracle.certify(enc, 1)[0] == oracle.ST_OK


@pytest.mark.parametrize("digit_bits", [8, 4])
def test_carry_matches_integer_value(digit_bits):
    rng = np.random.default_rng(9)
    for L in [1, 2, 10, 1000]:
        c = rng.integers(0, 5_000_000_000, L, dtype=np.int64)
        base = 1 << digit_bits
        value = sum(int(ci) * base ** i for i, ci in enumerate(c))
        nout = (L + 8) * digit_bits // 8 + 8
        out = oracle.carry(c, digit_bits, nout)
        assert int.from_bytes(out.tobytes(), "little") == value


# ---------------------------------------------------------------------------
# The paper's qualitative observations


def test_naive_single_precision_sometimes_wrong_at_120_digits():
    """Section 1: the naive (non-interval) single-precision variant is usually
    right but sometimes wrong for two 120-digit base-256 numbers."""
    wrong = 0
    trials = 150
    for s in range(trials):
        a, b = pair(1000 + s, 120)
        _, out = oracle.mul_naive(a, b, precision="f32")
        wrong += not np.array_equal(out, int_product(a, b))
    assert 0 < wrong < trials // 4


@pytest.mark.parametrize("n,kind", [(1024, "random"), (75000, "random"), (75000, "all_ff")])
def test_naive_double_matches_the_integer_product(n, kind):
    """The naive double-precision variant (section 3's "double naive" SSA) rounds
    every coefficient to the nearest integer without a certificate; at these
    sizes its rounding errors stay far below 1/2, so its products are exact."""
    a, b = pair(11, n) if kind == "random" else (np.full(n, 255, np.uint8), np.full(n, 255, np.uint8))
    st, out = oracle.mul_naive(a, b)
    assert st == oracle.ST_OK
    assert np.array_equal(out, int_product(a, b))
    st, out = oracle.mul_naive(a, b, digit_bits=4)
    assert np.array_equal(out, int_product(a, b))


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 16])
def test_naive_single_precision_exact_on_short_operands(n):
    """Short products (coefficients below 2^20, transforms of at most 32 points)
    leave single precision's rounding errors far below 1/2."""
    for s in range(40):
        a, b = pair(7000 + s, n)
        _, out = oracle.mul_naive(a, b, precision="f32")
        assert np.array_equal(out, int_product(a, b)), s
    f = np.full(n, 255, np.uint8)
    _, out = oracle.mul_naive(f, f, precision="f32")
    assert np.array_equal(out, int_product(f, f))


def test_single_precision_intervals_never_certify_a_wrong_product():
    for s in range(40):
        n = [8, 16, 24, 40, 64, 120][s % 6]
        a, b = pair(3000 + s, n)
        for bits in (8, 4):
            st, out, _, _ = oracle.mul(a, b, digit_bits=bits, precision="f32")
            if st == oracle.ST_OK:
                assert np.array_equal(out, int_product(a, b))
            else:
                assert st == oracle.ST_TOO_WIDE and not out.any()


# ---------------------------------------------------------------------------
# Planted mistakes: each plausible error in the oracle fails at least one pin.


def _pin_battery():
    """Runs a compact set of the pins above; returns the names that failed."""
    failed = []
    for a, b, c, z in read_tiny_products():
        st, out, _, _ = oracle.mul(a, b)
        if st != oracle.ST_OK or out.tolist() != z.tolist():
            failed.append("tiny")
            break
    a, b = pair(42, 300, 200)
    st, out, _, _ = oracle.mul(a, b)
    if st != oracle.ST_OK or not np.array_equal(out, int_product(a, b)):
        failed.append("product")
    try:
        test_dft_matches_definition_in_high_precision(3)
    except AssertionError:
        failed.append("dft")
    try:
        test_twiddles_contain_true_values(7)
    except AssertionError:
        failed.append("twiddle")
    try:
        test_directed_rounding_is_adjacent_f64("mul")
    except AssertionError:
        failed.append("rounding")
    return failed


def _naive_battery():
    """The naive variants' pins: double at 1024 bytes, single on short operands."""
    failed = []
    a, b = pair(11, 1024)
    if not np.array_equal(oracle.mul_naive(a, b)[1], int_product(a, b)):
        failed.append("naive_f64")
    a, b = pair(7000, 16)
    if not np.array_equal(oracle.mul_naive(a, b, precision="f32")[1], int_product(a, b)):
        failed.append("naive_f32")
    return failed


def test_planted_mistake_in_the_naive_variant_is_caught():
    """Mistake 9: the naive inverse transform keeps the forward roots."""
    assert _naive_battery() == []
    with oracle.mutation(9):
        failed = _naive_battery()
    assert failed == ["naive_f64", "naive_f32"], failed
    assert _naive_battery() == []


@pytest.mark.parametrize("mutation", [1, 2, 3, 4, 5, 6, 7, 8])
def test_planted_mistakes_are_caught(mutation):
    assert _pin_battery() == []
    with oracle.mutation(mutation):
        failed = _pin_battery()
    assert failed, "planted mistake %d went unnoticed" % mutation
    assert _pin_battery() == []
