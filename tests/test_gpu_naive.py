"""GPU tests of the non-rigorous point baseline (plan option arithmetic="naive").

The same kernels on plain complex doubles rounded to nearest, every coefficient
rounded to the nearest integer without a certificate: the naive method that
the paper's interval version is compared against (its section 3 times both).
Its products are checked against CPython's integers at sizes where double
precision is ample; its largest distance of a coefficient to its integer is
reported beside the rectangles' certified radius.
"""
import numpy as np
import pytest

from paper_1006_0405_amd import binding
from paper_1006_0405_amd.workloads import all_ff, pair
from pins import int_product

pytestmark = pytest.mark.gpu


def _np(t):
    return t.cpu().numpy()


@pytest.mark.parametrize("na,nb", [(1, 1), (100, 57), (1024, 1024), (2049, 2048), (6000, 3000),
                                   (30000, 29000), (75000, 75000)])
def test_naive_products_exact_where_doubles_suffice(na, nb):
    plan = binding.Plan(na, nb, arithmetic="naive")
    rect = binding.Plan(na, nb)
    for a, b in (pair(na + 3 * nb, na, nb), (all_ff(na), all_ff(nb))):
        st, out = plan.mul(a, b)
        assert st == binding.SSA_OK
        assert np.array_equal(_np(out), int_product(a, b)), (na, nb)
        d = plan.stats()["max_radius"]
        assert d < 0.5
        rect.mul(a, b)
        r = rect.stats()["max_radius"]
        print("%d x %d: naive distance to the integers %.3g, rectangle radius %.3g" % (na, nb, d, r))
    plan.close()
    rect.close()


def test_naive_batch_mixed_lengths():
    rng = np.random.default_rng(44)
    A, B = [], []
    for i in range(150):
        na = int(rng.integers(1, 12000))
        nb = int(rng.integers(1, 12000))
        a, b = pair(30_000 + i, na, nb)
        A.append(a)
        B.append(b)
    plan = binding.Plan(12000, 12000, arithmetic="naive")
    bt = binding.Batch(plan, A, B)
    st = _np(bt.run())
    assert np.all(st == binding.SSA_OK)
    for i in range(len(A)):
        assert np.array_equal(_np(bt.OUT[i]), int_product(A[i], B[i])), i
    bt.close()
    plan.close()


def test_naive_rejected_combinations():
    for kw in ({"precision": "fp32_fallback"}, {"separate_transforms": True},
               {"refine_digits": True}, {"refine_disc": True}):
        with pytest.raises(binding.SsaError):
            binding.Plan(5000, 5000, arithmetic="naive", **kw)
    plan = binding.Plan(30000, 30000, arithmetic="naive")
    log_n = binding.fft_size(30000, 30000).bit_length() - 1
    with pytest.raises(binding.SsaError):  # no persistent row pass
        plan.set_config(log_n, 8, 4, 1, 1)
    plan.close()


# ---- the single-precision naive baseline (arithmetic="naive32") -------------

def _naive32_wrong(n, count, seed0):
    """Products of `count` random n x n-byte pairs in naive FP32 (one batch):
    how many differ from the integer product, and the largest distance of a
    coefficient to its nearest integer."""
    A, B = [], []
    for i in range(count):
        a, b = pair(seed0 + i, n)
        A.append(a)
        B.append(b)
    plan = binding.Plan(n, n, arithmetic="naive32")
    bt = binding.Batch(plan, A, B)
    st = _np(bt.run())
    assert np.all(st == binding.SSA_OK)  # the run ended; no certificate
    wrong = sum(not np.array_equal(_np(bt.OUT[i]), int_product(A[i], B[i])) for i in range(count))
    dist = max(s["max_radius"] for s in bt.stats())
    bt.close()
    plan.close()
    return wrong, dist


def test_naive32_exact_for_short_operands():
    """A few bytes: single precision is ample (coefficients below 2^20)."""
    wrong, dist = _naive32_wrong(8, 512, 70_000)
    assert wrong == 0 and dist < 0.5
    plan = binding.Plan(16, 16, arithmetic="naive32")
    st, out = plan.mul(all_ff(16), all_ff(16))
    assert st == binding.SSA_OK and np.array_equal(_np(out), int_product(all_ff(16), all_ff(16)))
    plan.close()


def test_naive32_fails_where_single_precision_runs_out():
    """Section 1: the naive single-precision transform is usually right and
    sometimes wrong at 120 base-256 digits; longer operands are wrong almost
    always.  The share at 120 digits is reported, the trend checked."""
    w120, d120 = _naive32_wrong(120, 2048, 71_000)
    w1k, d1k = _naive32_wrong(1000, 256, 72_000)
    print("naive FP32 wrong products: 120 x 120 bytes %d of 2048 (%.2f%%, largest distance "
          "%.3g); 1000 x 1000 bytes %d of 256 (largest distance %.3g)"
          % (w120, 100.0 * w120 / 2048, d120, w1k, d1k))
    assert w1k > 128 and d1k >= 0.25  # distances to the nearest integer are at most 1/2
    assert 0 < w120 < 1024  # sometimes wrong, usually right at 120 digits (66 of 2048 measured)


def test_naive32_limits():
    with pytest.raises(binding.SsaError):  # beyond one workgroup's transform
        binding.Plan(2049, 2049, arithmetic="naive32")
    for kw in ({"precision": "fp32_fallback"}, {"refine_digits": True}, {"exact_fallback": True}):
        with pytest.raises(binding.SsaError):
            binding.Plan(100, 100, arithmetic="naive32", **kw)
