"""The exact last resort (plan option exact_fallback): when every interval run
refuses a product, ssa_mul computes it by a number-theoretic transform over
Z_p, p = 2^64 - 2^32 + 1 (section 1: another algorithm when the enclosures
are too wide; the paper's introduction: the second, finite-ring
Schoenhage-Strassen algorithm needs no approximation).

Its result has a plain definition, the exact product, so it is compared with
the integer product (CPython's, itself pinned to the oracle's long
multiplication on the CPU), with the oracle's certified product where the
oracle certifies, and with the closed form of (256^n - 1)(256^m - 1).  The
certification hook that refuses every interval enclosure sends products of
every length through it; a random 2 MiB product that the FP64 rectangles
really refuse, and products beyond the interval kernels' 2^22 points, go
through it without the hook.
"""
import numpy as np
import pytest
import torch

import oracle
from pins import all_ff_product, int_product, to_int
from paper_1006_0405_amd import binding
from paper_1006_0405_amd.workloads import all_ff, pair

pytestmark = pytest.mark.gpu

# (na, nb) covering transform lengths 2^9..2^20 (every remainder of log2 N mod
# 4, i.e. every last-pass radix) with ragged, tiny and very unequal operands
SIZES = [(1, 1), (1, 2000), (7, 300), (300, 17), (513, 511), (1024, 1024), (1500, 1049),
         (4096, 4095), (6000, 5000), (9000, 7385), (16384, 16384), (30000, 35000), (75000, 75000),
         (100000, 3), (200000, 100001), (400000, 300000)]


@pytest.fixture(scope="module")
def hooked_plan():
    plan = binding.Plan(400000, 300000, exact_fallback=True)
    plan.force_too_wide(True)  # every interval run refuses: the exact transform runs
    yield plan
    plan.close()


@pytest.mark.parametrize("na,nb", SIZES)
def test_exact_transform_gives_the_product(hooked_plan, na, nb):
    print("exact transform, random operands %d x %d" % (na, nb), flush=True)
    a, b = pair(9000 + na, na, nb)
    st, out = hooked_plan.mul(a, b)
    s = hooked_plan.stats()
    assert st == binding.SSA_OK and s["refined"] == 3 and s["max_radius"] == 0.0
    out = out.cpu().numpy()
    assert np.array_equal(out, int_product(a, b)), (na, nb)
    if na * nb <= 6000 * 5000:
        ost, oout, _, _ = oracle.mul(a, b)
        assert ost == oracle.ST_OK and np.array_equal(out, oout)


@pytest.mark.parametrize("na,nb", [(1, 1), (1024, 1024), (75000, 75000), (400000, 300000)])
def test_exact_transform_all_ff(hooked_plan, na, nb):
    print("exact transform, all-0xFF operands %d x %d" % (na, nb), flush=True)
    st, out = hooked_plan.mul(all_ff(na), all_ff(nb))
    assert st == binding.SSA_OK and hooked_plan.stats()["refined"] == 3
    assert np.array_equal(out.cpu().numpy(), all_ff_product(na, nb))


def test_exact_rung_takes_what_every_fp64_run_refuses():
    """Random 2 MiB operands (N = 2^22 in base 256): the rectangles refuse
    (radius about 4), and without the option the product is reported too
    wide; with it the exact transform returns the product."""
    n = 1 << 21
    print("2 MiB x 2 MiB random, base 256, no refinement", flush=True)
    a, b = pair(77, n)
    plain = binding.Plan(n, n)
    st, out = plain.mul(a, b)
    s = plain.stats()
    plain.close()
    assert st == binding.SSA_ENCLOSURE_TOO_WIDE and s["log_n"] == 22 and s["max_radius"] > 1
    assert not out.cpu().numpy().any()
    exact = binding.Plan(n, n, exact_fallback=True)
    st, out = exact.mul(a, b)
    s = exact.stats()
    exact.close()
    assert st == binding.SSA_OK and s["refined"] == 3
    assert np.array_equal(out.cpu().numpy(), int_product(a, b))


def _residue_checks(a, b, out):
    """The product modulo three 61-bit primes and its low 4096 bytes exactly."""
    A, B, Z = to_int(a), to_int(b), to_int(out)
    for q in (2305843009213693951, 2305843009213693921, 2305843009213693907):
        assert (A % q) * (B % q) % q == Z % q, q
    low = 4096
    want = (to_int(a[:low]) * to_int(b[:low])) % (256 ** low)
    assert to_int(out[:low]) == want


def test_exact_transform_beyond_the_interval_kernels():
    """Operands of 2^22 + 5 and 2^22 bytes: 2^23 + 4 coefficients, a transform
    of 2^24 points (the interval kernels stop at 2^22), straight to the exact
    transform."""
    na, nb = (1 << 22) + 5, 1 << 22
    print("exact transform beyond 2^22 points: %d x %d bytes" % (na, nb), flush=True)
    plan = binding.Plan(na, na, exact_fallback=True)
    a, b = pair(78, na, nb)
    st, out = plan.mul(a, b)
    s = plan.stats()
    assert st == binding.SSA_OK and s["refined"] == 3 and s["log_n"] == 24
    _residue_checks(a, b, out.cpu().numpy())
    st, out = plan.mul(all_ff(na), all_ff(na))
    assert st == binding.SSA_OK
    assert np.array_equal(out.cpu().numpy(), all_ff_product(na, na))
    plan.close()


def test_exact_fallback_plan_limits():
    with pytest.raises(binding.SsaError, match="INVALID_ARGUMENT"):
        binding.Plan(1 << 22, 1 << 22)  # 2^23 points, beyond the interval kernels
    with pytest.raises(binding.SsaError, match="INVALID_ARGUMENT"):
        binding.Plan(1 << 26, (1 << 26) + 2, exact_fallback=True)  # beyond 2^27 points
    with pytest.raises(binding.SsaError, match="INVALID_ARGUMENT"):
        binding.Plan(1000, 1000, arithmetic="naive", exact_fallback=True)
    # the exact plan's batches keep to the interval kernels' lengths
    na = (1 << 21) + 1
    plan = binding.Plan(na, na, exact_fallback=True)
    a = torch.zeros(na, dtype=torch.uint8, device="cuda")
    with pytest.raises(binding.SsaError, match="INVALID_ARGUMENT"):
        binding.Batch(plan, [a], [a])
    plan.close()
