"""CPU check of the FP64 disc (midpoint-radius) bounds used on the GPU.

The GPU's disc operations (circular containment sets, the paper's section 4)
compute a midpoint with operations rounded toward +infinity and grow the radius
by a bound of the roundings and of the input radii.  This test restates each
operation's formulas with directed rounding emulated exactly (Fractions, then
the smallest double not below the exact value) and checks, on random and
adversarial inputs, that the resulting disc contains the exact result for
points on the input discs' boundaries and roots of unity with rational
coordinates (Pythagorean triples: |w| = 1 exactly).
"""
import math
import random
from fractions import Fraction as F

U = F(1, 2 ** 52)
ETA = F(1, 2 ** 1074)


def ru(x):
    """The smallest double >= x (x a Fraction)."""
    d = float(x)
    if F(d) < x:
        d = math.nextafter(d, math.inf)
    return F(d)


# ---- the GPU formulas, each operation rounded up --------------------------

def md_add(a, b):
    re = ru(a[0] + b[0])
    im = ru(a[1] + b[1])
    r = ru(U * abs(re) + ru(U * abs(im) + ru(a[2] + b[2])))
    return re, im, r


def md_tw(a, c, s, e):
    p = ru(s * a[1])
    q = ru(c * a[1])
    re = ru(c * a[0] - p)
    im = ru(s * a[0] + q)
    k = ru(F(3, 2) * e + F(2.9) * U)  # the constants as the device holds them
    r = ru(k * abs(a[0]) + ru(k * abs(a[1]) + ru(a[2] + 8 * ETA)))
    return re, im, r


def md_mul(a, b):
    p1 = ru(a[1] * b[1])
    p2 = ru(a[1] * b[0])
    re = ru(a[0] * b[0] - p1)
    im = ru(a[0] * b[1] + p2)
    ma = ru(abs(a[0]) + abs(a[1]))
    mb = ru(abs(b[0]) + abs(b[1]))
    t = ru(F(2.0001) * U * mb + b[2])
    r = ru(ma * t + ru(a[2] * ru(mb + b[2]) + 8 * ETA))
    return re, im, r


# ---- checks -----------------------------------------------------------------

def inside(d, z):
    """|z - m| <= r, checked exactly (squares)."""
    dx, dy = z[0] - d[0], z[1] - d[1]
    return dx * dx + dy * dy <= d[2] * d[2]


def boundary_points(d, n=8):
    """Points of the disc: centre and n rational points near the boundary
    (scaled Pythagorean directions, modulus <= 1)."""
    dirs = [(F(3, 5), F(4, 5)), (F(-4, 5), F(3, 5)), (F(-3, 5), F(-4, 5)), (F(4, 5), F(-3, 5)),
            (F(5, 13), F(12, 13)), (F(-12, 13), F(5, 13)), (F(1), F(0)), (F(0), F(-1))]
    pts = [(d[0], d[1])]
    for ux, uy in dirs[:n]:
        pts.append((d[0] + d[2] * ux, d[1] + d[2] * uy))
    return pts


ROOTS = [(F(3, 5), F(4, 5)), (F(4, 5), F(3, 5)), (F(-5, 13), F(12, 13)), (F(-12, 13), F(-5, 13)),
         (F(8, 17), F(-15, 17)), (F(1), F(0)), (F(0), F(1)), (F(-20, 29), F(21, 29))]


def rand_disc(rng):
    scale = 2.0 ** rng.randint(-30, 40)
    re = F(rng.uniform(-1, 1) * scale)
    im = F(rng.uniform(-1, 1) * scale)
    r = F(abs(rng.uniform(0, 1)) * scale * 2.0 ** rng.randint(-60, -1)) if rng.random() < 0.9 else F(0)
    return re, im, r


def test_disc_add_contains_sums():
    rng = random.Random(1)
    for _ in range(300):
        a, b = rand_disc(rng), rand_disc(rng)
        c = md_add(a, b)
        for za in boundary_points(a, 4):
            for zb in boundary_points(b, 4):
                assert inside(c, (za[0] + zb[0], za[1] + zb[1]))


def test_disc_rotation_contains_rotated_points():
    rng = random.Random(2)
    for _ in range(300):
        a = rand_disc(rng)
        wt = rng.choice(ROOTS)
        # the stored point: the doubles nearest the root, and their error bound
        c, s = F(float(wt[0])), F(float(wt[1]))
        e = ru(max(abs(c - wt[0]), abs(s - wt[1])) + F(1, 2 ** 70))
        z = md_tw(a, c, s, e)
        for za in boundary_points(a):
            exact = (wt[0] * za[0] - wt[1] * za[1], wt[1] * za[0] + wt[0] * za[1])
            assert inside(z, exact)


def test_disc_rotation_with_a_perturbed_root():
    """The stored point may sit anywhere within e of the root in each
    component."""
    rng = random.Random(3)
    for _ in range(300):
        a = rand_disc(rng)
        wt = rng.choice(ROOTS)
        e = F(1, 2 ** rng.randint(20, 54))
        c = wt[0] + e * F(rng.choice([-1, 1]))
        s = wt[1] + e * F(rng.choice([-1, 1]))
        c, s = F(float(c)), F(float(s))
        e = ru(max(abs(c - wt[0]), abs(s - wt[1])))
        z = md_tw(a, c, s, e)
        for za in boundary_points(a):
            exact = (wt[0] * za[0] - wt[1] * za[1], wt[1] * za[0] + wt[0] * za[1])
            assert inside(z, exact)


def test_disc_product_contains_products():
    rng = random.Random(4)
    for _ in range(300):
        a, b = rand_disc(rng), rand_disc(rng)
        z = md_mul(a, b)
        for za in boundary_points(a, 4):
            for zb in boundary_points(b, 4):
                exact = (za[0] * zb[0] - za[1] * zb[1], za[0] * zb[1] + za[1] * zb[0])
                assert inside(z, exact)


def test_a_dropped_rounding_term_is_caught():
    """The checks above can fail: the rotation without its rounding terms
    (k = 1.5 e only) misses exact results for exact-point inputs."""
    rng = random.Random(5)
    missed = 0
    for _ in range(300):
        a = (F(rng.uniform(-1, 1) * 1e6), F(rng.uniform(-1, 1) * 1e6), F(0))
        wt = rng.choice(ROOTS[:5])
        c, s = F(float(wt[0])), F(float(wt[1]))
        e = ru(max(abs(c - wt[0]), abs(s - wt[1])))
        p, q = ru(s * a[1]), ru(c * a[1])
        re, im = ru(c * a[0] - p), ru(s * a[0] + q)
        k = ru(F(3, 2) * e)
        r = ru(k * abs(a[0]) + k * abs(a[1]))
        exact = (wt[0] * a[0] - wt[1] * a[1], wt[1] * a[0] + wt[0] * a[1])
        if not inside((re, im, r), exact):
            missed += 1
    assert missed > 0
