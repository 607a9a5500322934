"""GPU tests of the FP64 disc arithmetic (plan option arithmetic="disc").

Every product runs its FP64 transforms in midpoint-radius discs, the circular
containment sets of the paper's section 4, instead of rectangles: the
single-workgroup products (N <= 2^12) and the three passes above.  The product
must be the same exact integer: bit-exact against CPython's integers, the
oracle (which works in rectangles, the paper's section 2.5) and the all-0xFF
closed form; every enclosure must contain the exact convolution coefficient.  The disc and rectangle radii are reported side
by side.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1006_0405_amd import binding
from paper_1006_0405_amd.workloads import all_ff, pair
from pins import all_ff_product, exact_convolution, int_product, nibbles

pytestmark = pytest.mark.gpu


def _np(t):
    return t.cpu().numpy()


@pytest.mark.parametrize("na,nb", [(2049, 2048), (6000, 3000), (8192, 8192), (16384, 16384),
                                   (20000, 12000), (30000, 29000)])
def test_disc_products_vs_oracle(na, nb):
    a, b = pair(na + 5 * nb, na, nb)
    plan = binding.Plan(na, nb, arithmetic="disc")
    st, out = plan.mul(a, b)
    assert st == binding.SSA_OK, binding.STATUS_NAMES.get(st, st)
    out = _np(out)
    assert np.array_equal(out, int_product(a, b))
    ost, oout, orad, _ = oracle.mul(a, b)
    assert ost == oracle.ST_OK and np.array_equal(out, oout)
    print("%d x %d: disc radius %.3g, oracle (rectangles) %.3g" % (na, nb, plan.stats()["max_radius"],
                                                                  orad))
    plan.close()


@pytest.mark.parametrize("n", [75000, 131072])
def test_disc_2p18_random_and_all_ff_with_rect_radius(n):
    a, b = pair(2, n)
    f = all_ff(n)
    rads = {}
    for arith in ("rect", "disc"):
        plan = binding.Plan(n, n, arithmetic=arith)
        st, out = plan.mul(a, b)
        assert st == binding.SSA_OK
        assert np.array_equal(_np(out), int_product(a, b))
        rads[arith] = plan.stats()["max_radius"]
        st, out = plan.mul(f, f)
        assert st == binding.SSA_OK
        assert np.array_equal(_np(out), all_ff_product(n, n))
        rads[arith + "_ff"] = plan.stats()["max_radius"]
        plan.close()
    print("%d bytes, N = 2^18: radius rect %.4g / disc %.4g; all-0xFF rect %.4g / disc %.4g" % (
        n, rads["rect"], rads["disc"], rads["rect_ff"], rads["disc_ff"]))


@pytest.mark.parametrize("na,nb,digit_bits", [(9000, 7000, 8), (16000, 16384, 8), (5000, 4000, 4),
                                              (30000, 30000, 8)])
def test_disc_enclosures_contain_exact_coefficients(na, nb, digit_bits):
    a, b = pair(na * 3 + nb, na, nb)
    plan = binding.Plan(na, nb, digit_bits=digit_bits, arithmetic="disc")
    st, out, enc = plan.debug_enclosures(a, b)
    enc = _np(enc)
    assert st == binding.SSA_OK
    assert np.array_equal(_np(out), int_product(a, b))
    c = exact_convolution(a, b) if digit_bits == 8 else exact_convolution(nibbles(a), nibbles(b))
    L = len(c)
    assert np.all(enc[:, 0] <= enc[:, 1])
    assert np.all(enc[:L, 0] <= c) and np.all(c <= enc[:L, 1])
    assert np.all(enc[L:, 0] <= 0) and np.all(enc[L:, 1] >= 0)
    plan.close()


def test_disc_config5_base16_random_and_all_ff():
    n = 1_000_000
    plan = binding.Plan(n, n, digit_bits=4, arithmetic="disc")
    a, b = pair(5, n)
    st, out = plan.mul(a, b)
    assert st == binding.SSA_OK, binding.STATUS_NAMES.get(st, st)
    assert _np(out).tobytes() == (int.from_bytes(a.tobytes(), "little") *
                                  int.from_bytes(b.tobytes(), "little")).to_bytes(2 * n, "little")
    r = plan.stats()["max_radius"]
    f = all_ff(n)
    st, out = plan.mul(f, f)
    assert st == binding.SSA_OK
    assert np.array_equal(_np(out), all_ff_product(n, n))
    print("config5 disc: radius random %.4g, all-0xFF %.4g" % (r, plan.stats()["max_radius"]))
    plan.close()


def test_disc_every_plain_launch_shape():
    nbytes = 30000
    a, b = pair(nbytes + 17, nbytes, nbytes - 9)
    want = int_product(a, b)
    plan = binding.Plan(nbytes, nbytes, arithmetic="disc")
    log_n = binding.fft_size(nbytes, nbytes).bit_length() - 1
    tried = 0
    for l1 in range(6, 12):
        l2 = log_n - l1
        if not 6 <= l2 <= 11:
            continue
        for cols in (1, 2, 4, 8, 16, 32):
            for rows in (1, 2, 4, 8, 16, 32, 64):
                try:
                    plan.set_config(log_n, l1, cols, rows, 0)
                except binding.SsaError:
                    continue
                st, out = plan.mul(a, b)
                assert st == binding.SSA_OK, (l1, cols, rows)
                assert np.array_equal(_np(out), want), (l1, cols, rows)
                tried += 1
        with pytest.raises(binding.SsaError):  # no persistent row pass for discs
            plan.set_config(log_n, l1, 4, 1, 1)
    assert tried >= 8
    plan.close()


def test_disc_batch_mixed_lengths_and_autotuner():
    rng = np.random.default_rng(33)
    A, B = [], []
    for i in range(200):
        na = int(rng.integers(1, 12000))
        nb = int(rng.integers(1, 12000))
        if i % 7 == 3:
            A.append(all_ff(na))
            B.append(all_ff(nb))
        else:
            a, b = pair(20_000 + i, na, nb)
            A.append(a)
            B.append(b)
    plan = binding.Plan(12000, 12000, arithmetic="disc")
    res = plan.autotune(15, count=8)
    assert res["persistent"] == 0
    bt = binding.Batch(plan, A, B)
    st = _np(bt.run())
    assert np.all(st == binding.SSA_OK)
    for i in range(len(A)):
        assert np.array_equal(_np(bt.OUT[i]), int_product(A[i], B[i])), i
    bt.close()
    plan.close()


@pytest.mark.parametrize("digit_bits", [8, 4])
def test_disc_single_workgroup_products(digit_bits):
    sizes = [(1, 1), (1, 2), (3, 5), (17, 33), (100, 100), (127, 2), (255, 256), (511, 512),
             (1000, 1), (1023, 1025), (2048, 2048)]
    plan = binding.Plan(2048, 2048, digit_bits=digit_bits, arithmetic="disc")
    rect = binding.Plan(2048, 2048, digit_bits=digit_bits)
    for s, (na, nb) in enumerate(sizes):
        if digit_bits == 4 and na + nb > 2049:
            continue
        a, b = pair(900 + s, na, nb)
        st, out = plan.mul(a, b)
        assert st == binding.SSA_OK, (na, nb)
        assert np.array_equal(_np(out), int_product(a, b)), (na, nb)
        f = all_ff(na)
        st, out = plan.mul(f, f)
        assert st == binding.SSA_OK and np.array_equal(_np(out), int_product(f, f)), na
        rd = plan.stats()["max_radius"]
        rect.mul(f, f)
        print("%d x %d all-0xFF: radius disc %.3g, rect %.3g" % (na, na, rd, rect.stats()["max_radius"]))
    st, out, enc = plan.debug_enclosures(*pair(77, 1000, 900))
    enc = _np(enc)
    a, b = pair(77, 1000, 900)
    c = exact_convolution(a, b) if digit_bits == 8 else exact_convolution(nibbles(a), nibbles(b))
    assert st == binding.SSA_OK
    assert np.all(enc[:len(c), 0] <= c) and np.all(c <= enc[:len(c), 1])
    assert np.all(enc[:, 2] <= 0) and np.all(enc[:, 3] >= 0)
    plan.close()
    rect.close()


@pytest.mark.parametrize("digit_bits", [8, 4])
def test_disc_fp32_attempt_exact_and_fallback_counts(digit_bits):
    """The FP32 attempt's forward transform (FP32 discs) followed by the FP64
    product and inverse in discs instead of rectangles: products exact either
    way; how many sizes certify without the FP64 re-run is printed for both."""
    sizes = [(1, 1), (1, 2), (3, 5), (17, 33), (64, 65), (100, 100), (127, 2), (200, 57),
             (255, 256), (300, 300), (511, 512), (1000, 1), (1023, 1025)]
    used = {}
    for arith in ("rect", "disc"):
        plan = binding.Plan(2048, 2048, digit_bits=digit_bits, precision="fp32_fallback",
                            arithmetic=arith)
        plan.set_fp32_policy(4096)  # attempt FP32 on every single-workgroup product
        used[arith] = []
        for s, (na, nb) in enumerate(sizes):
            if digit_bits == 4 and na + nb > 2049:
                continue
            a, b = pair(700 + s, na, nb)
            st, out = plan.mul(a, b)
            assert st == binding.SSA_OK, (arith, na, nb)
            assert np.array_equal(_np(out), int_product(a, b)), (arith, na, nb)
            assert plan.stats()["fp32_attempt"] == 1
            used[arith].append(plan.stats()["fallback"])
        plan.close()
    print("FP32 attempts certified without re-run: rect %d, disc %d of %d" % (
        used["rect"].count(0), used["disc"].count(0), len(used["rect"])))


def test_refine_disc_rescues_a_product_too_wide_in_rectangles():
    """1 MiB random operands (N = 2^21): the rectangles hold several integers,
    the re-run in discs certifies the exact product (stats.refined = 2)."""
    n = 1 << 20
    a, b = pair(2, n)
    want = (int.from_bytes(a.tobytes(), "little") *
            int.from_bytes(b.tobytes(), "little")).to_bytes(2 * n, "little")
    plain = binding.Plan(n, n)
    st, out = plain.mul(a, b)
    assert st == binding.SSA_ENCLOSURE_TOO_WIDE
    assert not _np(out).any()
    plain.close()
    plan = binding.Plan(n, n, refine_disc=True)
    st, out = plan.mul(a, b)
    s = plan.stats()
    assert st == binding.SSA_OK and s["refined"] == 2
    assert _np(out).tobytes() == want
    print("1 MiB random: rectangles too wide, disc re-run radius %.4g" % s["max_radius"])
    c, d = pair(3, 5000)  # certified at once: no re-run
    st, out = plan.mul(c, d)
    assert st == binding.SSA_OK and plan.stats()["refined"] == 0
    assert np.array_equal(_np(out), int_product(c, d))
    plan.close()
    with pytest.raises(binding.SsaError):
        binding.Plan(5000, 5000, arithmetic="disc", refine_disc=True)
    with pytest.raises(binding.SsaError):
        binding.Plan(5000, 5000, separate_transforms=True, refine_disc=True)


def test_disc_rejected_with_separate_transforms():
    with pytest.raises(binding.SsaError):
        binding.Plan(5000, 5000, separate_transforms=True, arithmetic="disc")
    with pytest.raises(binding.SsaError):
        binding.Plan(5000, 5000, arithmetic="circle")
