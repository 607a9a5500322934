"""The device certification step against the oracle's (paper section 1: the
unique integer in each enclosure, else an error; the enclosures of section 2.5).

ssa_probe_certify runs the kernels' own certify()/cert_reduce() on enclosures
the test supplies.  Per entry, the outcome (one integer / several / impossible,
and whether the real part holds a half-integer) and the coefficient must equal
what oracle.certify gives for that entry alone; over the whole array, the
status, the largest radius (bit for bit) and the half-integer count must equal
the oracle's.  The table of certification cases derived from section 1 is also
checked against its stated outcomes directly.

The corrupted-bound hook (ssa_plan_corrupt_bound) drives the impossible-
enclosure branch through the real product kernels: the single-workgroup
kernel, the three-pass inverse column pass and a batch.
"""
import math

import numpy as np
import pytest

import oracle
from pins import int_product
from paper_1006_0405_amd import binding
from paper_1006_0405_amd.workloads import pair

pytestmark = pytest.mark.gpu

OK, WIDE, INTERNAL = 0, 1, 5

# (re_lo, re_hi), expected outcome, coefficient, half-integer inside.  The first
# six rows are the basic cases of section 1's rule on closed intervals (one
# integer inside, an exact integer, zero, a half-integer end point, two
# integers, none); the rest add the negative, tail and mixed cases.
TABLE = [
    ((2.6, 3.4), OK, 3, 0),
    ((3.0, 3.0), OK, 3, 0),
    ((-0.2, 0.3), OK, 0, 0),
    ((2.5, 3.5), OK, 3, 1),
    ((2.9, 4.1), WIDE, 0, 1),
    ((3.2, 3.8), INTERNAL, 0, 1),
    ((3.0, 3.9), OK, 3, 1),
    ((-1.2, -0.9), INTERNAL, 0, 0),
    ((-1.3, 5.0), WIDE, 0, 1),
    ((0.0, 0.0), OK, 0, 0),
    ((-0.5, 0.5), OK, 0, 1),
    ((2.0 ** 40, 2.0 ** 40), OK, 2 ** 40, 0),
]


def _oracle_entry(e, L, mode):
    """Outcome code of one entry as the probe encodes it, from the oracle."""
    st, c, rad, half = oracle.certify(e.reshape(1, 4), L, mode)
    return (st | (16 if half else 0)), (int(c[0]) if L else 0), rad


def _compare(enc, L, mode=binding.SSA_CERTIFY_ONE_INTEGER):
    """Probe vs oracle, entry by entry and in total."""
    enc = np.ascontiguousarray(enc, dtype=np.float64)
    n = enc.shape[0]
    st, c, cls = binding.probe_certify(enc, L, mode)
    ost, oc, orad, ohalf = oracle.certify(enc, L, mode)
    assert st["status"] == ost, (st, ost)
    assert st["max_radius"] == orad, (st["max_radius"], orad)  # bit for bit
    assert st["half_int"] == ohalf
    np.testing.assert_array_equal(c, oc)
    want = np.empty(n, dtype=np.int64)
    for i in range(n):
        code, _, _ = _oracle_entry(enc[i], 1 if i < L else 0, mode)
        want[i] = code
    bad = np.nonzero(cls != want)[0]
    assert bad.size == 0, [(int(i), enc[i].tolist(), int(cls[i]), int(want[i])) for i in bad[:10]]
    assert st["internal"] == int(np.sum((cls & 15) == INTERNAL))
    assert st["too_wide"] == int(np.sum((cls & 15) == WIDE))
    return st, c, cls


@pytest.mark.parametrize("case", TABLE, ids=lambda c: "%r" % (c[0],))
def test_certification_table(case):
    (lo, hi), outcome, value, half = case
    enc = np.array([[lo, hi, -1e-9, 1e-9]])
    st, c, cls = _compare(enc, 1)
    assert cls[0] == outcome | (16 * half)
    assert st["status"] == outcome
    assert c[0] == value
    assert st["max_radius"] >= (hi - lo) / 2


def test_strict_mode_refuses_half_integers():
    enc = np.array([[2.5, 3.5, 0.0, 0.0], [2.6, 3.4, 0.0, 0.0]])
    st, c, cls = _compare(enc, 2, binding.SSA_CERTIFY_HALF_INTEGER)
    assert st["status"] == WIDE and cls.tolist() == [WIDE | 16, OK]
    st, c, cls = _compare(enc, 2, binding.SSA_CERTIFY_ONE_INTEGER)
    assert st["status"] == OK and c.tolist() == [3, 3]


def test_imaginary_part_and_padded_tail():
    cases = [
        (np.array([[3.0, 3.0, 0.1, 0.2]]), 1, INTERNAL),     # imaginary part excludes 0
        (np.array([[3.0, 3.0, -0.2, -0.0]]), 1, OK),        # -0 still contains 0
        (np.array([[3.0, 3.0, 0, 0], [0.5, 0.6, 0, 0]]), 1, INTERNAL),   # tail excludes 0
        (np.array([[3.0, 3.0, 0, 0], [-0.5, 0.6, 0, 0]]), 1, OK),
        (np.array([[3.0, 3.0, 0, 0], [-0.5, 0.6, 0.1, 0.3]]), 1, INTERNAL),  # tail imag
        (np.array([[-3.0, 3.0, 0, 0], [-0.5, 0.6, 0, 0]]), 0, OK),  # all tail
    ]
    for enc, L, outcome in cases:
        st, _, _ = _compare(enc, L)
        assert st["status"] == outcome, enc


def _adversarial(rng, n):
    """Enclosures around integers of every magnitude the kernels can certify:
    bounds at k +- 1/2, one ulp either side of an integer, exact integers,
    random widths, negative centres, and imaginary parts that mostly (not
    always) contain 0."""
    mags = np.array([0, 1, 3, 255, 65025, 2.0 ** 20, 2.0 ** 32, 2.0 ** 40, 2.0 ** 48, 2.0 ** 51])
    k = np.floor(rng.random(n) * mags[rng.integers(0, len(mags), n)])
    k[rng.random(n) < 0.1] *= -1
    offs = np.array([-1.5, -1.0, -0.75, -0.5, -0.25, 0.0, 0.25, 0.5, 0.75, 1.0, 1.5])
    lo = k + offs[rng.integers(0, len(offs), n)]
    hi = k + offs[rng.integers(0, len(offs), n)]
    # ulp-adjacent bounds
    sel = rng.random(n) < 0.25
    lo[sel] = np.nextafter(k[sel], -np.inf)
    sel2 = rng.random(n) < 0.25
    hi[sel2] = np.nextafter(k[sel2], np.inf)
    sel3 = rng.random(n) < 0.1  # one ulp off a half-integer
    lo[sel3] = np.nextafter(k[sel3] + 0.5, np.where(rng.random(sel3.sum()) < 0.5, -np.inf, np.inf))
    # random widths
    sel4 = rng.random(n) < 0.25
    lo[sel4] = k[sel4] + rng.uniform(-1, 1, sel4.sum())
    hi[sel4] = lo[sel4] + rng.exponential(0.3, sel4.sum())
    lo, hi = np.minimum(lo, hi), np.maximum(lo, hi)
    t = rng.exponential(1e-6, n)
    im_lo, im_hi = -t, t
    sel5 = rng.random(n) < 0.02
    im_lo[sel5] = t[sel5]
    im_hi[sel5] = 2 * t[sel5] + 1e-9
    return np.stack([lo, hi, im_lo, im_hi], axis=1)


@pytest.mark.parametrize("mode", [binding.SSA_CERTIFY_ONE_INTEGER, binding.SSA_CERTIFY_HALF_INTEGER],
                         ids=["one_integer", "half_integer"])
def test_random_and_adversarial_enclosures(mode):
    rng = np.random.default_rng(20 + mode)
    n = 100_000
    enc = _adversarial(rng, n)
    L = n - 1000  # the last 1000 entries are a padded tail
    enc[L:, 0] = np.minimum(enc[L:, 0], 0.0)  # most tail entries contain 0 ...
    enc[L:, 1] = np.maximum(enc[L:, 1], 0.0)
    enc[L::97, 0] = 0.25                       # ... a few do not
    enc[L::97, 1] = 0.75
    st, c, cls = _compare(enc, L, mode)
    counts = {code: int(np.sum((cls & 15) == code)) for code in (OK, WIDE, INTERNAL)}
    print("outcomes over %d entries: %s, half-integers %d, max radius %r"
          % (n, counts, st["half_int"], st["max_radius"]))
    assert min(counts.values()) > 1000  # every branch is exercised many times


def test_each_coefficient_alone_certifies_when_valid():
    """A whole array of valid enclosures (radius < 1/2 around non-negative
    integers, imaginary parts holding 0) certifies with the exact integers."""
    rng = np.random.default_rng(7)
    n = 20_000
    k = rng.integers(0, 2 ** 40, n).astype(np.float64)
    r = rng.uniform(0, 0.49, n)
    enc = np.stack([k - r, k + r, -r, r], axis=1)
    st, c, _ = _compare(enc, n)
    assert st["status"] == OK
    np.testing.assert_array_equal(c, k.astype(np.int64))


def test_coefficients_of_2p52_and_beyond_are_impossible_on_the_device():
    """The device converts a certified coefficient through the binary64
    integers below 2^52 and reports a larger one as impossible (no product the
    library accepts has a coefficient above 2^40).  The oracle, which keeps
    such a value, differs only there."""
    enc = np.array([[2.0 ** 52, 2.0 ** 52, 0, 0]])
    st, c, cls = binding.probe_certify(enc, 1)
    assert st["status"] == INTERNAL and cls[0] == INTERNAL
    ost, oc, _, _ = oracle.certify(enc, 1)
    assert ost == OK and oc[0] == 2 ** 52


def test_probe_rejects_bad_arguments():
    enc = np.zeros((4, 4))
    with pytest.raises(binding.SsaError):
        binding.probe_certify(enc, 5)  # L > n
    with pytest.raises(binding.SsaError):
        binding.probe_certify(enc, 2, mode=7)


# ---------------------------------------------------------------------------
# The impossible-enclosure branch through the product kernels.


def _np(t):
    return t.cpu().numpy()


@pytest.mark.parametrize("na,nb,digit_bits", [(1024, 1024, 8), (300, 200, 4), (6000, 5000, 8),
                                               (40000, 30000, 8), (3000, 2500, 4)])
def test_corrupted_bound_reports_internal_error(na, nb, digit_bits):
    a, b = pair(77, na, nb)
    plan = binding.Plan(na, nb, digit_bits=digit_bits)
    L = (na + nb) * (2 if digit_bits == 4 else 1) - 1
    for idx in (0, 1, L // 2, L - 1):
        plan.corrupt_bound(idx)
        st, out = plan.mul(a, b)
        s = plan.stats()
        assert st == binding.SSA_INTERNAL_ERROR, (idx, binding.STATUS_NAMES.get(st))
        assert s["internal"] == 1 and s["too_wide"] == 0, (idx, s)
        assert not _np(out).any(), "output not zero-filled"
    plan.corrupt_bound(L + 5)  # a padded-tail index: no coefficient is touched
    st, out = plan.mul(a, b)
    assert st == binding.SSA_OK and np.array_equal(_np(out), int_product(a, b))
    plan.corrupt_bound(-1)
    st, out = plan.mul(a, b)
    assert st == binding.SSA_OK and np.array_equal(_np(out), int_product(a, b))
    plan.close()


def test_corrupted_bound_in_a_batch():
    pairs = [pair(500 + i, n, m) for i, (n, m) in enumerate([(100, 90), (2000, 2048), (9000, 7000),
                                                              (30000, 20000), (700, 800)])]
    A, B = [p[0] for p in pairs], [p[1] for p in pairs]
    plan = binding.Plan(max(map(len, A)), max(map(len, B)))
    plan.corrupt_bound(3)
    bt = binding.Batch(plan, A, B)
    status = _np(bt.run())
    assert np.all(status == binding.SSA_INTERNAL_ERROR), status
    assert all(s["internal"] == 1 for s in bt.stats())
    assert not any(_np(o).any() for o in bt.OUT)
    bt.close()
    plan.corrupt_bound(-1)
    bt = binding.Batch(plan, A, B)
    status = _np(bt.run())
    assert np.all(status == binding.SSA_OK)
    for a, b, o in zip(A, B, bt.OUT):
        assert np.array_equal(_np(o), int_product(a, b))
    bt.close()
    plan.close()


def test_corrupt_hook_arguments():
    plan = binding.Plan(10, 10)
    for bad in (-2, 1 << 31):
        with pytest.raises(binding.SsaError):
            plan.corrupt_bound(bad)
    plan.close()


def test_half_integer_count_of_a_product_matches_the_oracle_on_thin_enclosures():
    """Products whose enclosures are tiny: no coefficient enclosure holds a
    half-integer on either side."""
    a, b = pair(5, 1024)
    plan = binding.Plan(1024, 1024)
    st, out = plan.mul(a, b)
    s = plan.stats()
    ost, oout, orad, ohalf = oracle.mul(a, b)
    assert st == ost == binding.SSA_OK
    assert s["half_int"] == ohalf == 0
    assert math.isfinite(s["max_radius"]) and s["max_radius"] < 0.5
    print("max radius: GPU %r, oracle %r" % (s["max_radius"], orad))
    plan.close()
