"""GPU parity tests: the HIP library through its C ABI against the oracle.

Products are integers, so the bar is bit-exact equality with the oracle's
product and with CPython's integer product (and schoolbook / closed forms where
they apply).  Enclosures are not unique; they are checked by containment of
the exact coefficients, and the GPU's maximum radius is reported next to the
oracle's.  Directed rounding is checked bit-for-bit against exact rationals.
"""
import math
from fractions import Fraction

import mpmath
import numpy as np
import pytest
import torch

import oracle
from paper_1006_0405_amd import binding
from paper_1006_0405_amd.workloads import all_ff, batch, pair
from pins import (all_ff_coefficients, all_ff_product, exact_convolution, int_product,
                  long_multiplication, nibbles)

pytestmark = pytest.mark.gpu


def _np(t):
    return t.cpu().numpy()


def _round_down(q):
    f = float(q)
    if Fraction(f) > q:
        f = float(np.nextafter(f, -np.inf))
    return f


def _round_up(q):
    f = float(q)
    if Fraction(f) < q:
        f = float(np.nextafter(f, np.inf))
    return f


# ---------------------------------------------------------------------------
# Directed rounding primitives (section 2.5: outward rounding)


def test_directed_rounding_bit_exact():
    rng = np.random.default_rng(17)
    n = 4000
    a = rng.standard_normal(n) * np.exp2(rng.integers(-40, 40, n))
    b = rng.standard_normal(n) * np.exp2(rng.integers(-40, 40, n))
    c = rng.standard_normal(n) * np.exp2(rng.integers(-40, 40, n))
    edge = np.array([0.0, -0.0, 1.0, -1.0, 0.5, 3.0, 1e-310, -1e-310, 5e-324, 2.0 ** 52,
                     2.0 ** 53 - 1, 1.0 + 2.0 ** -52, 0.1, -0.7, 123456789.123, 1e-300])
    a[:len(edge)] = edge
    b[:len(edge)] = edge[::-1]
    c[:len(edge)] = np.roll(edge, 3)
    exact = {
        0: lambda x, y, z: Fraction(x) + Fraction(y),
        1: lambda x, y, z: Fraction(x) * Fraction(y),
        2: lambda x, y, z: Fraction(x) * Fraction(y) + Fraction(z),
    }
    for op in range(6):
        got = _np(binding.probe_directed(op, a, b, c))
        f = exact[op % 3]
        rnd = _round_up if op < 3 else _round_down
        for i in range(n):
            want = rnd(f(a[i], b[i], c[i]))
            assert got[i] == want or (got[i] == 0 and want == 0), (op, a[i], b[i], c[i], got[i], want)


# ---------------------------------------------------------------------------
# Twiddles (section 2.2 recurrence, computed on the device)


def _omega_iv(m, N):
    m %= N
    if (4 * m) % N == 0:
        q = 4 * m // N
        return [(mpmath.iv.mpf(x), mpmath.iv.mpf(y)) for x, y in [(1, 0), (0, 1), (-1, 0), (0, -1)]][q]
    ang = 2 * mpmath.iv.pi * m / N
    return mpmath.iv.cos(ang), mpmath.iv.sin(ang)


@pytest.mark.parametrize("nbytes", [1000, 75000])
def test_twiddle_table_encloses_roots_of_unity(nbytes):
    plan = binding.Plan(nbytes, nbytes)
    tab, e, lg = plan.twiddles()
    plan.close()
    tab = _np(tab)
    N = 1 << lg
    # half an ulp of the stored midpoint plus the fixed-point enclosure width
    # (about 2^-62 per exact product over the set bits of t): below one ulp of 1
    print("twiddle table 2^%d: e = %.3e" % (lg, e))
    assert 0 < e < 1.2e-16
    mpmath.iv.prec = 200
    idx = sorted(set([0, 1, N // 8, N // 4, N // 2, N - 1] + list(range(0, N, max(1, N // 700)))))
    for t in idx:
        cs, sn = _omega_iv(t, N)
        for val, iv in ((tab[t, 0], cs), (tab[t, 1], sn)):
            lo, hi = mpmath.mpf(val) - mpmath.mpf(e), mpmath.mpf(val) + mpmath.mpf(e)
            assert lo <= iv.a and iv.b <= hi, (t, val, iv, e)


# ---------------------------------------------------------------------------
# Single products


def _check_product(plan, a, b, digit_bits=8, with_oracle=True):
    st, out = plan.mul(a, b)
    out = _np(out)
    assert st == binding.SSA_OK, binding.STATUS_NAMES.get(st, st)
    assert np.array_equal(out, int_product(a, b))
    if with_oracle:
        ost, oout, orad, _ = oracle.mul(a, b, digit_bits=digit_bits)
        assert ost == oracle.ST_OK
        assert np.array_equal(out, oout)
    return out


def test_tiny_products():
    from test_oracle import read_tiny_products
    plan = binding.Plan(8, 8)
    for a, b, c, z in read_tiny_products():
        st, out = plan.mul(a, b)
        assert st == binding.SSA_OK
        assert _np(out).tolist() == z.tolist()
    plan.close()


@pytest.mark.parametrize("separate", [False, True], ids=["packed", "separate"])
@pytest.mark.parametrize("digit_bits", [8, 4])
def test_small_path_ragged_sizes(digit_bits, separate):
    plan = binding.Plan(2048, 2048, digit_bits=digit_bits, separate_transforms=separate)
    sizes = [(1, 1), (1, 2), (2, 1), (3, 5), (17, 33), (64, 65), (127, 2), (128, 129), (200, 57),
             (255, 256), (511, 512), (1000, 1), (1023, 1025), (2048, 2048), (1500, 300)]
    for s, (na, nb) in enumerate(sizes):
        if digit_bits == 4 and na + nb > 2049:
            continue
        a, b = pair(500 + s, na, nb)
        _check_product(plan, a, b, digit_bits)
    plan.close()


def test_leading_zeros_and_zero_operands():
    plan = binding.Plan(300, 300)
    rng = np.random.default_rng(3)
    a = rng.integers(0, 256, 300, dtype=np.uint8)
    a[-40:] = 0
    z = np.zeros(100, np.uint8)
    for x, y in [(a, z), (z, a), (a, a), (z, z)]:
        _check_product(plan, x, y)
    plan.close()


def test_config1_product_vs_oracle_and_schoolbook():
    a, b = pair(1, 1024)
    plan = binding.Plan(1024, 1024)
    out = _check_product(plan, a, b)
    assert np.array_equal(out, long_multiplication(a, b))
    rad = plan.stats()["max_radius"]
    _, _, orad, _ = oracle.mul(a, b)
    print("config1: GPU max radius %.3e, oracle %.3e" % (rad, orad))
    assert 0 < rad < 0.5
    plan.close()


@pytest.mark.parametrize("separate", [False, True], ids=["packed", "separate"])
@pytest.mark.parametrize("na,nb,digit_bits", [(1, 1, 8), (300, 200, 8), (1024, 1024, 8),
                                              (2048, 2047, 8), (3000, 2500, 8), (5000, 9000, 8),
                                              (16000, 16384, 8), (700, 900, 4), (9000, 7000, 4)])
def test_enclosures_contain_exact_coefficients(na, nb, digit_bits, separate):
    a, b = pair(na * 7 + nb, na, nb)
    plan = binding.Plan(na, nb, digit_bits=digit_bits, separate_transforms=separate)
    st, out, enc = plan.debug_enclosures(a, b)
    enc = _np(enc)
    assert st == binding.SSA_OK
    assert np.array_equal(_np(out), int_product(a, b))
    if digit_bits == 8:
        c = exact_convolution(a, b)
    else:
        c = exact_convolution(nibbles(a), nibbles(b))
    L = len(c)
    assert np.all(enc[:, 0] <= enc[:, 1]) and np.all(enc[:, 2] <= enc[:, 3])
    assert np.all(enc[:L, 0] <= c) and np.all(c <= enc[:L, 1])
    assert np.all(enc[:, 2] <= 0) and np.all(enc[:, 3] >= 0)
    assert np.all(enc[L:, 0] <= 0) and np.all(enc[L:, 1] >= 0)
    plan.close()


@pytest.mark.parametrize("separate", [False, True], ids=["packed", "separate"])
@pytest.mark.parametrize("na,nb", [(2049, 2048), (4096, 4096), (6000, 3000), (8192, 8192),
                                   (16384, 16384), (20000, 12000)])
def test_multipass_products_vs_oracle(na, nb, separate):
    a, b = pair(na + 3 * nb, na, nb)
    plan = binding.Plan(na, nb, separate_transforms=separate)
    _check_product(plan, a, b)
    plan.close()


@pytest.mark.parametrize("n,m", [(2049, 2049), (8192, 100), (40000, 40000)])
def test_all_ff_multipass(n, m):
    plan = binding.Plan(n, m)
    st, out = plan.mul(all_ff(n), all_ff(m))
    assert st == binding.SSA_OK
    assert np.array_equal(_np(out), all_ff_product(n, m))
    plan.close()


@pytest.mark.parametrize("separate", [False, True], ids=["packed", "separate"])
def test_config2_random_and_all_ff(separate):
    n = 75000
    plan = binding.Plan(n, n, separate_transforms=separate)
    a, b = pair(2, n)
    st, out = plan.mul(a, b)
    out = _np(out)
    rad = plan.stats()["max_radius"]
    assert st == binding.SSA_OK
    assert np.array_equal(out, int_product(a, b))
    ost, oout, orad, _ = oracle.mul(a, b)
    assert ost == oracle.ST_OK and np.array_equal(out, oout)
    print("config2 random (%s): GPU max radius %.4f, oracle %.4f"
          % ("separate" if separate else "packed", rad, orad))
    assert 0 < rad <= orad  # radix-8 stages round less often than the oracle's radix-2 ones
    f = all_ff(n)
    st, out = plan.mul(f, f)
    assert st == binding.SSA_OK
    assert np.array_equal(_np(out), all_ff_product(n, n))
    print("config2 all-0xFF: GPU max radius %.4f" % plan.stats()["max_radius"])
    plan.close()


@pytest.mark.parametrize("separate", [False, True], ids=["packed", "separate"])
def test_config5_base16_random_and_all_ff(separate):
    n = 1_000_000
    plan = binding.Plan(n, n, digit_bits=4, separate_transforms=separate)
    a, b = pair(5, n)
    st, out = plan.mul(a, b)
    assert st == binding.SSA_OK, binding.STATUS_NAMES.get(st, st)
    assert _np(out).tobytes() == (int.from_bytes(a.tobytes(), "little") *
                                  int.from_bytes(b.tobytes(), "little")).to_bytes(2 * n, "little")
    print("config5 random: GPU max radius %.4f, log_n %d" % (plan.stats()["max_radius"],
                                                              plan.stats()["log_n"]))
    f = all_ff(n)
    st, out = plan.mul(f, f)
    assert st == binding.SSA_OK
    assert np.array_equal(_np(out), all_ff_product(n, n))
    print("config5 all-0xFF: GPU max radius %.4f" % plan.stats()["max_radius"])
    plan.close()


def test_config5_enclosures_contain_sampled_coefficients():
    n = 1_000_000
    plan = binding.Plan(n, n, digit_bits=4)
    a, b = pair(5, n)
    st, _, enc = plan.debug_enclosures(a, b)
    assert st == binding.SSA_OK
    x = nibbles(a).astype(np.int64)
    y = nibbles(b).astype(np.int64)
    L = len(x) + len(y) - 1
    rng = np.random.default_rng(0)
    idx = np.concatenate([[0, 1, L // 2, L - 2, L - 1], rng.integers(0, L, 1000)])
    enc_np = _np(enc[torch_index(idx)])
    for k, i in enumerate(idx):
        j0, j1 = max(0, i - len(y) + 1), min(len(x) - 1, i)
        ci = int(np.dot(x[j0:j1 + 1], y[i - j1:i - j0 + 1][::-1]))
        assert enc_np[k, 0] <= ci <= enc_np[k, 1], (i, ci, enc_np[k])
    plan.close()


def torch_index(idx):
    import torch
    return torch.as_tensor(np.asarray(idx, dtype=np.int64), device="cuda")


def test_determinism():
    a, b = pair(77, 30000, 29000)
    plan = binding.Plan(30000, 29000)
    outs, rads = [], []
    for _ in range(3):
        st, out = plan.mul(a, b)
        assert st == binding.SSA_OK
        outs.append(_np(out))
        rads.append(plan.stats()["max_radius"])
    assert all(np.array_equal(outs[0], o) for o in outs[1:])
    assert rads[0] == rads[1] == rads[2]
    plan.close()


def test_invalid_arguments():
    plan = binding.Plan(100, 100)
    with pytest.raises(binding.SsaError):
        plan.mul(np.zeros(0, np.uint8), np.ones(3, np.uint8))
    with pytest.raises(binding.SsaError):
        plan.mul(np.ones(101, np.uint8), np.ones(3, np.uint8))
    plan.close()
    with pytest.raises(binding.SsaError):
        binding.Plan(0, 10)


def test_strict_half_integer_mode_never_wrong():
    plan = binding.Plan(5000, 5000, certify_mode=binding.SSA_CERTIFY_HALF_INTEGER)
    for s in range(4):
        a, b = pair(900 + s, 5000)
        st, out = plan.mul(a, b)
        assert st in (binding.SSA_OK, binding.SSA_ENCLOSURE_TOO_WIDE)
        if st == binding.SSA_OK:
            assert np.array_equal(_np(out), int_product(a, b))
        else:
            assert not _np(out).any()
    plan.close()


def test_too_wide_status_zero_fills_output():
    """The failure contract: a product whose enclosures are refused reports
    SSA_ENCLOSURE_TOO_WIDE and an all-zero output, on the single-workgroup path,
    the multi-pass path (carry scan) and in a batch; normal certification
    returns afterwards."""
    plan = binding.Plan(40000, 40000)
    cases = [pair(31, 1000, 700), pair(32, 40000, 39000), (all_ff(20000), all_ff(20000))]
    plan.force_too_wide(True)
    for a, b in cases:
        out = torch.full((len(a) + len(b),), 0xAB, dtype=torch.uint8, device="cuda")
        st, out = plan.mul(a, b, out=out)
        assert st == binding.SSA_ENCLOSURE_TOO_WIDE
        assert not _np(out).any()
        assert plan.stats()["too_wide"] > 0
    bt = binding.Batch(plan, [c[0] for c in cases], [c[1] for c in cases])
    for o in bt.OUT:
        o.fill_(0xCD)
    assert np.all(_np(bt.run()) == binding.SSA_ENCLOSURE_TOO_WIDE)
    assert all(not _np(o).any() for o in bt.OUT)
    bt.close()
    plan.force_too_wide(False)
    for a, b in cases:
        st, out = plan.mul(a, b)
        assert st == binding.SSA_OK and np.array_equal(_np(out), int_product(a, b))
    rc = binding.lib().ssa_plan_force_too_wide(plan.handle, 2)
    assert rc == binding.SSA_INVALID_ARGUMENT
    plan.close()


@pytest.mark.parametrize("n", [1 << 20])
def test_refine_digits_rescues_base256(n):
    """A random base-256 product beyond the FP64 frontier (1 MiB operands,
    N = 2^21) is refused in base 256; a plan with refine_digits re-runs it with
    base-16 digits (N = 2^22) and returns the exact product.  A product that
    certifies in base 256 is not re-run; with every enclosure refused both runs
    fail and the output is all zeros."""
    a, b = pair(2, n)
    plain = binding.Plan(n, n)
    st, _ = plain.mul(a, b)
    assert st == binding.SSA_ENCLOSURE_TOO_WIDE and plain.stats()["refined"] == 0
    plain.close()
    plan = binding.Plan(n, n, refine_digits=True)
    st, out = plan.mul(a, b)
    s = plan.stats()
    print("refined:", s)
    assert st == binding.SSA_OK and s["refined"] == 1 and s["log_n"] == 22
    assert np.array_equal(_np(out), int_product(a, b))
    c, d = pair(3, 70000)
    st, out = plan.mul(c, d)
    assert st == binding.SSA_OK and plan.stats()["refined"] == 0
    assert np.array_equal(_np(out), int_product(c, d))
    plan.force_too_wide(True)
    st, out = plan.mul(c, d)
    assert st == binding.SSA_ENCLOSURE_TOO_WIDE and plan.stats()["refined"] == 1
    assert not _np(out).any()
    plan.close()
    with pytest.raises(binding.SsaError):
        binding.Plan(100, 100, digit_bits=4, refine_digits=True)


def test_largest_transform_base256():
    """The largest transform a plan accepts (2^22) with base-256 digits: 2 MiB
    operands (beyond the FP64 certification frontier for random bytes: the
    enclosures are refused); certified products are exact, a refused one is all
    zeros, and operands one byte longer are rejected at plan creation."""
    n = 1 << 21
    a, b = pair(77, n)
    plan = binding.Plan(n, n)
    st, out = plan.mul(a, b)
    s = plan.stats()
    print("2^22 base 256: status", st, "radius", s["max_radius"])
    assert s["log_n"] == 22
    if st == binding.SSA_OK:
        assert np.array_equal(_np(out), int_product(a, b))
    else:
        assert st == binding.SSA_ENCLOSURE_TOO_WIDE and not _np(out).any()
    plan.close()
    with pytest.raises(binding.SsaError):
        binding.Plan(n + 1, n + 1)  # L = 2^22 + 1 needs a transform of 2^23


# ---------------------------------------------------------------------------
# Batches


def test_batch_mixed_lengths():
    rng = np.random.default_rng(21)
    A, B = [], []
    for i in range(300):
        na = int(rng.integers(1, 12000))
        nb = int(rng.integers(1, 12000))
        a, b = pair(10_000 + i, na, nb)
        A.append(a)
        B.append(b)
    plan = binding.Plan(12000, 12000)
    bt = binding.Batch(plan, A, B)
    for rep in range(2):
        status = _np(bt.run())
        assert np.all(status == binding.SSA_OK)
        for i in range(len(A)):
            assert np.array_equal(_np(bt.OUT[i]), int_product(A[i], B[i])), i
    st = bt.stats()
    assert all(s["status"] == 0 for s in st)
    bt.close()
    plan.close()


def test_config3_batch_full():
    A, B = batch(seed=3)
    plan = binding.Plan(16384, 16384)
    bt = binding.Batch(plan, A, B)
    status = _np(bt.run())
    assert np.all(status == binding.SSA_OK)
    for i in range(len(A)):
        assert np.array_equal(_np(bt.OUT[i]), int_product(A[i], B[i])), i
    rads = [s["max_radius"] for s in bt.stats()]
    print("config3: %d products, max radius %.4f" % (len(A), max(rads)))
    bt.close()
    plan.close()


# ---------------------------------------------------------------------------
# Launch shapes: products do not depend on the shape; the autotuner's choice is valid


def _valid_shapes(log_n, packed=True):
    out = []
    for l1 in range(6, 12):
        l2 = log_n - l1
        if not 6 <= l2 <= 11:
            continue
        for cols in (1, 2, 4, 8, 16, 32):
            for rows in (1, 2, 4, 8, 16, 32, 64):
                ct = cols * (1 << l1) // 8
                rt = (2 if packed else 1) * rows * (1 << l2) // 8
                pad1 = (1 << l1) + (1 << l1) // 8
                pad2 = (1 << l2) + (1 << l2) // 8
                if (ct > 512 or ct % 64 or pad1 * cols * 16 > 81920 or (1 << l2) // 2 % cols
                        or rt > 512 or rt % 64 or (2 if packed else 1) * rows * pad2 * 16 > 81920
                        or ((1 << l1) // 2 if packed else (1 << l1)) % rows):
                    continue
                out.append((l1, cols, rows, 0))
                # the persistent row pass: packed rows of at most 2^9 points, with the
                # twiddle levels up to 2^l2 in LDS beside the exchange buffers
                if packed and l2 <= 9 and (2 * rows * pad2 + (2 << l2)) * 16 <= 81920:
                    out.append((l1, cols, rows, 1))
    return out


@pytest.mark.parametrize("separate", [False, True], ids=["packed", "separate"])
@pytest.mark.parametrize("nbytes", [5000, 30000])
def test_every_launch_shape_gives_the_same_product(nbytes, separate):
    a, b = pair(nbytes + 11, nbytes, nbytes - 7)
    plan = binding.Plan(nbytes, nbytes, separate_transforms=separate)
    log_n = binding.fft_size(nbytes, nbytes).bit_length() - 1
    want = int_product(a, b)
    shapes = _valid_shapes(log_n, packed=not separate)
    assert len(shapes) >= 4
    for l1, cols, rows, pers in shapes:
        plan.set_config(log_n, l1, cols, rows, pers)
        assert plan.get_config(log_n) == {"log_n1": l1, "cols": cols, "rows": rows,
                                          "persistent": pers, "inv_cols": cols}
        st, out = plan.mul(a, b)
        assert st == binding.SSA_OK, (l1, cols, rows, pers)
        assert np.array_equal(_np(out), want), (l1, cols, rows, pers)
    with pytest.raises(binding.SsaError):
        plan.set_config(log_n, 3, 1, 1)
    with pytest.raises(binding.SsaError):
        plan.set_config(log_n, log_n // 2, 3, 1)
    with pytest.raises(binding.SsaError):
        plan.set_config(log_n, 6, 8, 1, 2)  # persistent flag out of range
    with pytest.raises(binding.SsaError):
        plan.set_config(log_n, shapes[0][0], shapes[0][1], shapes[0][2], 0, 3)  # inv_cols not 2^k
    plan.close()


@pytest.mark.parametrize("nbytes", [5000, 30000, 75000])
def test_inverse_column_count_gives_the_same_product(nbytes):
    """The inverse column pass with its own column count (every valid one), the
    other passes fixed: random and all-0xFF operands, all exact."""
    plan = binding.Plan(nbytes, nbytes)
    log_n = binding.fft_size(nbytes, nbytes).bit_length() - 1
    l1 = log_n // 2
    N1, N2 = 1 << l1, 1 << (log_n - l1)
    a, b = pair(nbytes + 5, nbytes, nbytes - 3)
    f = all_ff(nbytes)
    want_ab, want_ff = int_product(a, b), int_product(f, f)
    cols = 4 if N1 <= 1024 else 2
    rows = max(1, 32 // (N2 // 8))  # row-pair workgroups of whole wavefronts
    tried = 0
    for ic in (1, 2, 4, 8, 16, 32):
        if ic * N1 // 8 > 512 or ic * N1 // 8 % 64 or (N1 + N1 // 8) * ic * 16 > 81920 or (N2 // 2) % ic:
            with pytest.raises(binding.SsaError):
                plan.set_config(log_n, l1, cols, rows, 0, ic)
            continue
        plan.set_config(log_n, l1, cols, rows, 0, ic)
        assert plan.get_config(log_n)["inv_cols"] == ic
        for x, y, want in ((a, b, want_ab), (f, f, want_ff)):
            st, out = plan.mul(x, y)
            assert st == binding.SSA_OK, ic
            assert np.array_equal(_np(out), want), ic
        tried += 1
    assert tried >= 2
    plan.close()


@pytest.mark.parametrize("log_n,nbytes,shape", [(18, 75000, (9, 4, 1, 1)), (18, 75000, (9, 2, 2, 1)),
                                               (14, 5000, (7, 8, 4, 1)), (16, 30000, (7, 4, 2, 1))])
def test_persistent_row_pass_batch(log_n, nbytes, shape):
    """Batches long enough that every persistent row-pass workgroup walks several
    items (prefetching the next while computing the current), products in
    descending order: random, all-0xFF and ragged operands, all exact."""
    plan = binding.Plan(nbytes, nbytes)
    assert binding.fft_size(nbytes, nbytes).bit_length() - 1 == log_n
    plan.set_config(log_n, *shape)
    A, B = [], []
    for i in range(40):
        if i % 3 == 1:
            A.append(all_ff(nbytes))
            B.append(all_ff(nbytes - 5 * i))
        else:
            a, b = pair(900 + i, nbytes - 3 * i, nbytes - 7 * (i % 5))
            A.append(a)
            B.append(b)
    assert all(binding.fft_size(len(a), len(b)).bit_length() - 1 == log_n for a, b in zip(A, B))
    bt = binding.Batch(plan, A, B)
    st = _np(bt.run())
    assert np.all(st == binding.SSA_OK)
    for i in range(len(A)):
        assert np.array_equal(_np(bt.OUT[i]), int_product(A[i], B[i])), i
    bt.close()
    plan.close()


def test_autotuner_choice_is_used_and_correct(tmp_path):
    n = 75000
    plan = binding.Plan(n, n)
    cache = str(tmp_path / "tune.json")
    res = plan.autotune(18, count=8, cache=cache)
    assert not res["cached"] and res["tried"] >= 4 and res["ms_per_batch"] > 0
    print("autotune 2^18:", res)
    again = plan.autotune(18, count=8, cache=cache)
    assert again["cached"] and again["log_n1"] == res["log_n1"]
    assert plan.get_config(18) == {k: res[k] for k in ("log_n1", "cols", "rows", "persistent",
                                                       "inv_cols")}
    a, b = pair(2, n)
    st, out = plan.mul(a, b)
    assert st == binding.SSA_OK and np.array_equal(_np(out), int_product(a, b))
    plan.close()
