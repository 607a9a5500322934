"""CPU check of the FP32 disc (midpoint-radius) bounds of the single-precision
first attempt.

The GPU's FP32 discs (circular containment sets, the paper's section 4, in the
reduced precision its section 1 speaks of) compute a midpoint in FP32 with
round-to-nearest and grow the radius by a bound of what the midpoint lost.
This test restates each operation's formulas with FP32 round-to-nearest-even
emulated exactly (Fractions, then the nearest float32, ties to even, with
subnormals), in the order the device evaluates them and also with the radius
sums fused into one multiply-add where the compiler may contract them, and
checks that the disc contains the exact result for points on the input discs'
boundaries.  Roots of unity with rational coordinates (Pythagorean triples,
|w| = 1 exactly) stand in for the twiddles; the length-8 butterfly with its
irrational root (1 + i)/sqrt 2 is checked against 200-bit values.  A rotation
without its rounding terms must fail the same checks.
"""
import random
from fractions import Fraction as F

import mpmath

U = F(1, 2 ** 24)
ETA = F(1, 2 ** 126)
MIN_SUB = F(1, 2 ** 149)


def rn32(x):
    """The float32 nearest the Fraction x, ties to even (subnormals included)."""
    if x == 0:
        return F(0)
    s = -1 if x < 0 else 1
    a = abs(x)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if F(2) ** e > a:
        e -= 1
    assert F(2) ** e <= a < F(2) ** (e + 1)
    q = F(2) ** (max(e, -126) - 23)
    n = a / q
    fl = n.numerator // n.denominator
    rem = n - fl
    if rem > F(1, 2) or (rem == F(1, 2) and fl % 2 == 1):
        fl += 1
    assert fl * q < F(2) ** 128, "overflow"
    return s * fl * q


def f32(v):
    """A Python float as the float32 the device holds (a constant's rounding)."""
    return rn32(F(v))


# the constants as the device holds them
MR_U = f32(5.9604644775390625e-08)
MR_ETA = f32(1.1754943508222875e-38)
MR_UP = f32(1.0) + 8 * MR_U
MR_E32 = f32(5.9604651880817983e-08)
assert MR_U == U and MR_ETA == ETA and MR_UP == 1 + F(1, 2 ** 21)
assert MR_E32 == U * (1 + F(1, 2 ** 23))


# ---- the device formulas, each FP32 operation rounded to nearest ------------

def rad_sum(terms, scaled, extra, fused):
    """sum(terms) + MR_U * scaled + extra, then * MR_UP: left to right, or with
    the MR_U product fused into the addition that follows it."""
    t = terms[0]
    for x in terms[1:]:
        t = rn32(t + x)
    t = rn32(MR_U * scaled + t) if fused else rn32(t + rn32(MR_U * scaled))
    t = rn32(t + extra)
    return rn32(t * MR_UP)


def mr_add(a, b, fused=False, sign=1):
    re = rn32(a[0] + sign * b[0])
    im = rn32(a[1] + sign * b[1])
    r = rad_sum([a[2], b[2]], rn32(abs(re) + abs(im)), rn32(2 * MR_ETA), fused)
    return re, im, r


def mr_sub(a, b, fused=False):
    return mr_add(a, b, fused, -1)


def mr_mul_i(a):
    return -a[1], a[0], a[2]


def mr_tw(a, c, s, e, fused=False, drop_round=False):
    p = rn32(s * a[1])
    q = rn32(c * a[1])
    re = rn32(c * a[0] - p)  # fmaf(c, a.re, -p)
    im = rn32(s * a[0] + q)  # fmaf(s, a.re, q)
    absum = rn32(rn32(rn32(abs(re) + abs(im)) + abs(p)) + abs(q))
    rnd = rn32(MR_U * absum + 4 * MR_ETA) if fused else rn32(rn32(MR_U * absum) + rn32(4 * MR_ETA))
    k1 = rn32(1 + rn32(2 * e))   # (1.0f + 2.0f * e), folded to a float constant
    k2 = rn32(F(3, 2) * e)       # 1.5f * e
    mag = rn32(rn32(abs(a[0]) + abs(a[1])) + a[2])
    if fused:
        t = rn32(k2 * mag + rn32(k1 * a[2]))
    else:
        t = rn32(rn32(k1 * a[2]) + rn32(k2 * mag))
    if not drop_round:
        t = rn32(t + rnd)
    return re, im, rn32(t * MR_UP)


# ---- checks -------------------------------------------------------------------

def inside(d, z):
    """|z - m| <= r, exactly (squares)."""
    dx, dy = z[0] - d[0], z[1] - d[1]
    return dx * dx + dy * dy <= d[2] * d[2]


DIRS = [(F(3, 5), F(4, 5)), (F(-4, 5), F(3, 5)), (F(-3, 5), F(-4, 5)), (F(4, 5), F(-3, 5)),
        (F(5, 13), F(12, 13)), (F(-12, 13), F(5, 13)), (F(1), F(0)), (F(0), F(-1))]


def boundary_points(d, n=8):
    pts = [(d[0], d[1])]
    for ux, uy in DIRS[:n]:
        pts.append((d[0] + d[2] * ux, d[1] + d[2] * uy))
    return pts


ROOTS = [(F(3, 5), F(4, 5)), (F(4, 5), F(3, 5)), (F(-5, 13), F(12, 13)), (F(-12, 13), F(-5, 13)),
         (F(8, 17), F(-15, 17)), (F(1), F(0)), (F(0), F(1)), (F(-20, 29), F(21, 29))]


def rand_disc(rng, thin=0.1):
    """FP32 midpoint and radius over a wide range of magnitudes (integers up to
    2^24 as the digit transforms hold them, and fractions); a share are exact
    points (r = 0), where the rounding terms alone must cover the error."""
    scale = 2.0 ** rng.randint(-20, 40)
    re = rn32(F(rng.uniform(-1, 1) * scale))
    im = rn32(F(rng.uniform(-1, 1) * scale))
    r = F(0) if rng.random() < thin else rn32(F(rng.uniform(0, 1) * scale * 2.0 ** rng.randint(-30, -1)))
    return re, im, r


def test_rn32_emulation():
    """The emulated rounding against known float32 facts."""
    assert rn32(F(1) + F(1, 2 ** 24)) == 1                    # tie to even (down)
    assert rn32(F(1) + F(3, 2 ** 24)) == 1 + F(1, 2 ** 22)    # tie to even (up)
    assert rn32(F(1) + F(1, 2 ** 24) + F(1, 2 ** 60)) == 1 + F(1, 2 ** 23)
    assert rn32(MIN_SUB * F(3, 2)) == 2 * MIN_SUB             # subnormal tie to even
    assert rn32(F(1, 3)) == F(11184811, 2 ** 25)
    assert rn32(F(-16777217)) == -16777216


def test_fp32_disc_add_and_sub_contain_sums():
    rng = random.Random(11)
    for fused in (False, True):
        for _ in range(150):
            a, b = rand_disc(rng), rand_disc(rng)
            c, d = mr_add(a, b, fused), mr_sub(a, b, fused)
            for za in boundary_points(a, 4):
                for zb in boundary_points(b, 4):
                    assert inside(c, (za[0] + zb[0], za[1] + zb[1]))
                    assert inside(d, (za[0] - zb[0], za[1] - zb[1]))


def test_fp32_disc_rotation_contains_rotated_points():
    """The stored twiddle is the FP32 rounding of a root (mr_tw_tab: the double
    table entry converted to float), within MR_E32 of the root."""
    rng = random.Random(12)
    for fused in (False, True):
        for _ in range(200):
            a = rand_disc(rng, thin=0.3)
            wt = rng.choice(ROOTS)
            c, s = rn32(wt[0]), rn32(wt[1])
            assert abs(c - wt[0]) <= MR_E32 and abs(s - wt[1]) <= MR_E32
            z = mr_tw(a, c, s, MR_E32, fused)
            for za in boundary_points(a):
                exact = (wt[0] * za[0] - wt[1] * za[1], wt[1] * za[0] + wt[0] * za[1])
                assert inside(z, exact)


def test_fp32_disc_rotation_with_a_perturbed_root():
    """Any stored point within MR_E32 of the root in each component (the
    double table's own error plus the conversion to float)."""
    rng = random.Random(13)
    for _ in range(300):
        a = rand_disc(rng, thin=0.3)
        wt = rng.choice(ROOTS)
        c = rn32(wt[0] + MR_E32 * F(rng.uniform(-1, 1)))
        s = rn32(wt[1] + MR_E32 * F(rng.uniform(-1, 1)))
        if abs(c - wt[0]) > MR_E32 or abs(s - wt[1]) > MR_E32:
            continue
        z = mr_tw(a, c, s, MR_E32, fused=rng.random() < 0.5)
        for za in boundary_points(a):
            exact = (wt[0] * za[0] - wt[1] * za[1], wt[1] * za[0] + wt[0] * za[1])
            assert inside(z, exact)


def mr_radix4(v, fused):
    a, b = mr_add(v[0], v[2], fused), mr_sub(v[0], v[2], fused)
    c, d = mr_add(v[1], v[3], fused), mr_sub(v[1], v[3], fused)
    i_d = mr_mul_i(d)
    return [mr_add(a, c, fused), mr_add(b, i_d, fused), mr_sub(a, c, fused), mr_sub(b, i_d, fused)]


def mr_radix8(v, c8, fused):
    """The device's length-8 DFT (omega_8 = e^{+2 pi i/8}) as two length-4 DFTs."""
    a = [mr_add(v[r], v[r + 4], fused) for r in range(4)]
    b = [mr_sub(v[r], v[r + 4], fused) for r in range(4)]
    b[1] = mr_tw(b[1], c8, c8, MR_E32, fused)
    b[2] = mr_mul_i(b[2])
    b[3] = mr_tw(b[3], -c8, c8, MR_E32, fused)
    a, b = mr_radix4(a, fused), mr_radix4(b, fused)
    out = [None] * 8
    for m in range(4):
        out[2 * m], out[2 * m + 1] = a[m], b[m]
    return out


def test_fp32_radix8_contains_the_exact_dft():
    """Outputs enclose the length-8 DFT sum_n x_n omega_8^{nk} of points of
    the input discs, evaluated with 200-bit arithmetic (the margin tested is
    far above 2^-190 relative)."""
    mpmath.mp.prec = 200
    c8 = rn32(F(float(mpmath.sqrt(2) / 2)))  # the double table entry, as float
    w = [mpmath.expjpi(mpmath.mpf(2 * k) / 8) for k in range(8)]
    rng = random.Random(14)
    for trial in range(40):
        fused = trial % 2 == 1
        v = [rand_disc(rng, thin=0.5) for _ in range(8)]
        out = mr_radix8(v, c8, fused)
        for d in range(3):  # centres, and two boundary directions
            pts = [boundary_points(x)[0 if d == 0 else 2 * d] for x in v]
            xs = [mpmath.mpc(mpmath.mpf(p[0].numerator) / p[0].denominator,
                             mpmath.mpf(p[1].numerator) / p[1].denominator) for p in pts]
            for k in range(8):
                X = mpmath.fsum(xs[n] * w[(n * k) % 8] for n in range(8))
                m = out[k]
                mre = mpmath.mpf(m[0].numerator) / m[0].denominator
                mim = mpmath.mpf(m[1].numerator) / m[1].denominator
                r = mpmath.mpf(m[2].numerator) / m[2].denominator
                dist = mpmath.sqrt((X.real - mre) ** 2 + (X.imag - mim) ** 2)
                assert dist <= r * (1 - mpmath.mpf(2) ** -190), (trial, k, float(dist), float(r))


def test_a_dropped_rounding_term_is_caught():
    """The checks above can fail: the rotation without its rounding term, with
    the root's own error as its bound (no slack left in e), misses exact
    results for exact-point inputs."""
    rng = random.Random(15)
    missed = 0
    for _ in range(300):
        a = (rn32(F(rng.randint(-2 ** 24, 2 ** 24))), rn32(F(rng.randint(-2 ** 24, 2 ** 24))), F(0))
        wt = rng.choice(ROOTS[:5])
        c, s = rn32(wt[0]), rn32(wt[1])
        e = max(abs(c - wt[0]), abs(s - wt[1]))
        z = mr_tw(a, c, s, e, drop_round=True)
        exact = (wt[0] * a[0] - wt[1] * a[1], wt[1] * a[0] + wt[0] * a[1])
        if not inside(z, exact):
            missed += 1
    assert missed > 0


def test_a_halved_addition_rounding_term_is_caught():
    """The sum's checks can fail too: with half of its rounding term (and
    neither ETA nor the inflation) the disc of a sum of exact points misses the
    exact sum."""
    rng = random.Random(16)
    missed = 0
    for _ in range(400):
        a = (rn32(F(rng.randint(1, 2 ** 24))), rn32(F(rng.randint(1, 2 ** 24))), F(0))
        b = (rn32(F(rng.random())), rn32(F(rng.random())), F(0))
        re, im = rn32(a[0] + b[0]), rn32(a[1] + b[1])
        r = rn32(F(1, 2) * rn32(U * rn32(abs(re) + abs(im))))
        if not inside((re, im, r), (a[0] + b[0], a[1] + b[1])):
            missed += 1
    assert missed > 0
