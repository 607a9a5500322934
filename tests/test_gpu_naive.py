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
