"""CPU check that the first radix-8 stage of a digit transform computed on
exact points (radix8_thin in the kernels) gives the same enclosures as the
interval radix-8 stage on the thin rectangles of those digits.

Both device formulas are restated with every operation rounded toward
+infinity exactly (Fractions, then the smallest double not below).  Digits are
small integers, so the stage's sums and differences are exact and only the
products by omega_8 = c8 (1 + i) and omega_8^3 = c8 (-1 + i) round; the two
forms must agree bound for bound (zero bounds compared by value), and a
planted mistake in the point form (a swapped sign in the i b2 term) must show.
"""
import math
import random
from fractions import Fraction as F

C8 = F(0.7071067811865476)  # the stored omega_8 real part
E8 = F(1, 2 ** 53)


def ru(x):
    d = float(x)
    if F(d) < x:
        d = math.nextafter(d, math.inf)
    return F(d)


# ---- rectangles (rn, rh, in, ih), lower bounds negated ----------------------

def add(a, b):
    return tuple(ru(p + q) for p, q in zip(a, b))


def sub(a, b):
    return (ru(a[0] + b[1]), ru(a[1] + b[0]), ru(a[2] + b[3]), ru(a[3] + b[2]))


def mul_i(a):
    return (a[3], a[2], a[0], a[1])


def mul_w8(z):
    un, uh = ru(z[0] + z[3]), ru(z[1] + z[2])
    wn, wh = ru(z[0] + z[2]), ru(z[1] + z[3])
    eu, ew = ru(E8 * max(un, uh)), ru(E8 * max(wn, wh))
    return (ru(C8 * un + eu), ru(C8 * uh + eu), ru(C8 * wn + ew), ru(C8 * wh + ew))


def mul_w83(z):
    un, uh = ru(z[0] + z[3]), ru(z[1] + z[2])
    wn, wh = ru(z[0] + z[2]), ru(z[1] + z[3])
    eu, ew = ru(E8 * max(un, uh)), ru(E8 * max(wn, wh))
    return (ru(C8 * wh + ew), ru(C8 * wn + ew), ru(C8 * un + eu), ru(C8 * uh + eu))


def radix4(v):
    a, b = add(v[0], v[2]), sub(v[0], v[2])
    c, d = add(v[1], v[3]), sub(v[1], v[3])
    idd = mul_i(d)
    return [add(a, c), add(b, idd), sub(a, c), sub(b, idd)]


def radix8(v):
    a = [add(v[r], v[r + 4]) for r in range(4)]
    b = [sub(v[r], v[r + 4]) for r in range(4)]
    b[1], b[2], b[3] = mul_w8(b[1]), mul_i(b[2]), mul_w83(b[3])
    a, b = radix4(a), radix4(b)
    out = [None] * 8
    for m in range(4):
        out[2 * m], out[2 * m + 1] = a[m], b[m]
    return out


# ---- the point form ---------------------------------------------------------

def thin(x, y):
    return (-x, x, -y, y)


def radix8_thin(x, y, planted=False):
    ax = [ru(x[r] + x[r + 4]) for r in range(4)]
    ay = [ru(y[r] + y[r + 4]) for r in range(4)]
    bx = [ru(x[r] - x[r + 4]) for r in range(4)]
    by = [ru(y[r] - y[r + 4]) for r in range(4)]
    Ax, Ay = ru(ax[0] + ax[2]), ru(ay[0] + ay[2])
    Bx, By = ru(ax[0] - ax[2]), ru(ay[0] - ay[2])
    Cx, Cy = ru(ax[1] + ax[3]), ru(ay[1] + ay[3])
    Dx, Dy = ru(ax[1] - ax[3]), ru(ay[1] - ay[3])
    u1, w1 = ru(bx[1] - by[1]), ru(bx[1] + by[1])
    eu1, ew1 = ru(E8 * abs(u1)), ru(E8 * abs(w1))
    B1 = (ru(-C8 * u1 + eu1), ru(C8 * u1 + eu1), ru(-C8 * w1 + ew1), ru(C8 * w1 + ew1))
    u3, w3 = ru(bx[3] - by[3]), ru(bx[3] + by[3])
    eu3, ew3 = ru(E8 * abs(u3)), ru(E8 * abs(w3))
    B3 = (ru(C8 * w3 + ew3), ru(-C8 * w3 + ew3), ru(-C8 * u3 + eu3), ru(C8 * u3 + eu3))
    sgn = -1 if planted else 1
    Px, Py = ru(bx[0] - sgn * by[2]), ru(by[0] + sgn * bx[2])
    Qx, Qy = ru(bx[0] + sgn * by[2]), ru(by[0] - sgn * bx[2])
    C = add(B1, B3)
    D = mul_i(sub(B1, B3))
    v = [None] * 8
    v[0] = thin(ru(Ax + Cx), ru(Ay + Cy))
    v[4] = thin(ru(Ax - Cx), ru(Ay - Cy))
    v[2] = thin(ru(Bx - Dy), ru(By + Dx))
    v[6] = thin(ru(Bx + Dy), ru(By - Dx))
    v[1] = add(thin(Px, Py), C)
    v[5] = sub(thin(Px, Py), C)
    v[3] = add(thin(Qx, Qy), D)
    v[7] = sub(thin(Qx, Qy), D)
    return v


def digits(rng, top):
    return [F(rng.randrange(top)) for _ in range(8)]


def test_point_form_equals_the_interval_stage():
    rng = random.Random(11)
    for t in range(600):
        top = (256, 16, 2)[t % 3]
        x = digits(rng, top)
        y = digits(rng, top) if t % 4 else [F(0)] * 8  # separate transforms: real input
        want = radix8([thin(x[r], y[r]) for r in range(8)])
        got = radix8_thin(x, y)
        assert got == want, (x, y)


def test_planted_sign_mistake_shows():
    rng = random.Random(12)
    differs = 0
    for _ in range(100):
        x, y = digits(rng, 256), digits(rng, 256)
        want = radix8([thin(x[r], y[r]) for r in range(8)])
        differs += radix8_thin(x, y, planted=True) != want
    assert differs > 0
