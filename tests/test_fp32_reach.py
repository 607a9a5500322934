"""How far a rigorous single-precision transform reaches on the base-16 batch.

The paper's section 1 notes that a naive single-precision SSA is already
sometimes wrong at 120 base-256 digits, and that a failed certificate means
more precision is needed.  This CPU emulation asks how many products of the
4096-product base-16 batch (operand lengths log-uniform in 64..16,384 bytes)
a rigorous FP32 forward transform could certify at all.

The emulation runs the FP32 disc operations of the GPU's first attempt (sum,
difference and rotation by a twiddle, with their radius formulas and
constants) in numpy float32, which rounds to nearest like the device, over a
radix-2 transform of the packed digits z = a + i b.  The rest is taken in its
most favourable form: the separated pointwise product and the inverse in exact
arithmetic on the discs, so that the coefficient radius is
(1/N) sum_k (|A_k| r_B + |B_k| r_A + r_A r_B), the radius every output of a
disc inverse transform carries, without any rounding of its own.  The real
path only adds to this.  A product can certify only if that radius is below
1, and certifies for sure below 1/2.
"""
import numpy as np
import pytest

from paper_1006_0405_amd.workloads import batch_lengths, pair

U = np.float32(2.0 ** -24)
ETA2 = np.float32(2.0 * 2.0 ** -126)
ETA4 = np.float32(4.0 * 2.0 ** -126)
UP = np.float32(1.0 + 2.0 ** -21)
E32 = np.float32(2.0 ** -24 * (1.0 + 2.0 ** -23))
K1 = np.float32(1.0) + np.float32(2.0) * E32
K2 = np.float32(1.5) * E32


def _add(are, aim, ar, bre, bim, br, sign):
    re = are + sign * bre
    im = aim + sign * bim
    r = (((ar + br) + U * (np.abs(re) + np.abs(im))) + ETA2) * UP
    return re, im, r


def _tw(are, aim, ar, c, s):
    p = s * aim
    q = c * aim
    # fmaf(c, a.re, -p) and fmaf(s, a.re, q): one rounding of the exact value
    re = (c.astype(np.float64) * are.astype(np.float64) - p.astype(np.float64)).astype(np.float32)
    im = (s.astype(np.float64) * are.astype(np.float64) + q.astype(np.float64)).astype(np.float32)
    rnd = U * (((np.abs(re) + np.abs(im)) + np.abs(p)) + np.abs(q)) + ETA4
    r = ((K1 * ar + K2 * ((np.abs(are) + np.abs(aim)) + ar)) + rnd) * UP
    return re, im, r


def fp32_forward(z):
    """Radix-2 decimation-in-time DFT (omega = e^{+2 pi i/N}) of thin discs
    z (complex digits), with the device's FP32 disc operations."""
    N = len(z)
    log_n = N.bit_length() - 1
    rev = np.zeros(N, dtype=np.int64)
    for b in range(log_n):
        rev |= ((np.arange(N) >> b) & 1) << (log_n - 1 - b)
    re = z.real[rev].astype(np.float32)
    im = z.imag[rev].astype(np.float32)
    r = np.zeros(N, dtype=np.float32)
    for s in range(1, log_n + 1):
        m = 1 << s
        h = m >> 1
        ang = 2.0 * np.pi * np.arange(h) / m
        c = np.cos(ang).astype(np.float32)   # the double table entry, to float
        sn = np.sin(ang).astype(np.float32)
        re = re.reshape(-1, m)
        im = im.reshape(-1, m)
        r = r.reshape(-1, m)
        tre, tim, tr = _tw(re[:, h:], im[:, h:], r[:, h:], c[None, :], sn[None, :])
        ure, uim, ur = re[:, :h], im[:, :h], r[:, :h]
        sre, sim, sr = _add(ure, uim, ur, tre, tim, tr, 1)
        dre, dim_, dr = _add(ure, uim, ur, tre, tim, tr, -1)
        re = np.concatenate([sre, dre], axis=1).ravel()
        im = np.concatenate([sim, dim_], axis=1).ravel()
        r = np.concatenate([sr, dr], axis=1).ravel()
    return re.astype(np.float64) + 1j * im.astype(np.float64), r.astype(np.float64)


def nibbles(x):
    d = np.empty(2 * len(x), dtype=np.float64)
    d[0::2] = x & 15
    d[1::2] = x >> 4
    return d


def coefficient_radius(a, b):
    """The smallest coefficient radius an FP32 forward transform leaves (see
    the module docstring), for byte operands a and b in base-16 digits."""
    da, db = nibbles(a), nibbles(b)
    L = len(da) + len(db) - 1
    N = max(1 << int(np.ceil(np.log2(L))), 512)
    z = np.zeros(N, dtype=np.complex128)
    z.real[:len(da)] = da
    z.imag[:len(db)] = db
    Z, rz = fp32_forward(z)
    neg = (-np.arange(N)) % N
    A = (Z + np.conj(Z[neg])) / 2
    B = (Z - np.conj(Z[neg])) / 2j
    rA = (rz + rz[neg]) / 2
    return float(np.mean(np.abs(A) * rA + np.abs(B) * rA + rA * rA)), N


def test_fp32_reach_matches_the_measured_frontier():
    """Random operands filling a transform of 512 points certify (the GPU's
    FP32 attempt does, at L <= 511 nibbles); at 2048 points even this
    favourable radius is far above 1/2."""
    r512, n = coefficient_radius(*pair(7, 128))
    assert n == 512 and r512 < 0.5, r512
    r2k, n = coefficient_radius(*pair(7, 512))
    assert n == 2048 and r2k > 1.0, r2k
    print("FP32 forward transform, random bytes: radius %.3g at N = 512, %.3g at N = 2048"
          % (r512, r2k))


@pytest.mark.parametrize("sample", [256])
def test_fp32_reach_on_the_base16_batch(sample):
    """Per length class of the base-16 batch: the median radius over sampled
    products, and the share of the whole batch whose class certifies.  Below
    half of the batch can certify, so a rigorous FP32 forward transform cannot
    carry most of it; the products it reaches are the shortest ones."""
    _, na, nb = batch_lengths()
    L = 2 * na + 2 * nb - 1
    cls = np.maximum(np.ceil(np.log2(L)).astype(int), 9)
    rng = np.random.default_rng(99)
    idx = rng.choice(len(L), sample, replace=False)
    rows, certifiable = [], 0
    radius = {}
    for i in idx:
        a = rng.integers(0, 256, int(na[i]), dtype=np.uint8)
        b = rng.integers(0, 256, int(nb[i]), dtype=np.uint8)
        a[-1] = max(a[-1], 1)
        b[-1] = max(b[-1], 1)
        r, N = coefficient_radius(a, b)
        radius.setdefault(N, []).append(r)
    for N in sorted(radius):
        med = float(np.median(radius[N]))
        share = float(np.mean(np.array(radius[N]) < 0.5))
        count = int(np.sum(cls == N.bit_length() - 1))
        certifiable += share * count
        rows.append("N=%6d products %4d sampled %3d median radius %9.3g certify %.2f"
                    % (N, count, len(radius[N]), med, share))
    print("\n".join(rows))
    print("batch share an FP32 forward transform can certify: %.3f" % (certifiable / len(L)))
    assert certifiable / len(L) < 0.5
    assert min(radius) == 512 and np.median(radius[512]) < 0.5
