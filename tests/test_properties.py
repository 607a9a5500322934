"""Property-based tests (hypothesis): operands of arbitrary lengths and bytes,
including the edge cases a fixed list misses (leading zero bytes, zero
operands, one-byte operands, lengths one past a power of two).

CPU (the oracle, which the GPU tests then trust):
  * the oracle's certified product equals CPython's integer product, in both
    digit sizes; a refused product is all zeros and never wrong;
  * every exact convolution coefficient lies inside its enclosure (section
    2.5: the enclosures are rigorous);
  * the oracle's carry loop reproduces the integer from arbitrary
    coefficients below 2^40 (section 2.4's carry box);
  * long multiplication (the LM box pin) equals the integer product.
GPU (marked gpu): ssa_mul, the batch path, the exact last resort and long
multiplication on generated operands, against the integer product and, for
ssa_mul, against the oracle's status.
"""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings, strategies as st

import oracle
from pins import exact_convolution, int_product, long_multiplication, nibbles, to_int

operand = st.binary(min_size=1, max_size=300).map(lambda b: np.frombuffer(b, dtype=np.uint8).copy())
special = st.sampled_from(["random", "zeros", "ff", "one"])


def shaped(data, kind):
    if kind == "zeros":
        return np.zeros_like(data)
    if kind == "ff":
        return np.full_like(data, 0xFF)
    if kind == "one":
        z = np.zeros_like(data)
        z[0] = 1
        return z
    return data


CPU = settings(max_examples=120, deadline=None, suppress_health_check=[HealthCheck.too_slow])


@CPU
@given(operand, operand, special, special, st.sampled_from([8, 4]))
def test_oracle_product_is_the_integer_product(a, b, ka, kb, bits):
    a, b = shaped(a, ka), shaped(b, kb)
    st_, out, rad, _ = oracle.mul(a, b, digit_bits=bits)
    if st_ == oracle.ST_OK:
        assert np.array_equal(out, int_product(a, b))
        assert rad < 1.0
    else:
        assert st_ == oracle.ST_TOO_WIDE and not out.any()


@CPU
@given(operand, operand, st.sampled_from([8, 4]))
def test_oracle_enclosures_contain_the_exact_coefficients(a, b, bits):
    enc = oracle.conv_enclosure(a, b, digit_bits=bits)
    da, db = (a, b) if bits == 8 else (nibbles(a), nibbles(b))
    c = exact_convolution(da, db).astype(np.float64)
    N = enc.shape[0]
    full = np.zeros(N)
    full[:len(c)] = c
    assert np.all(enc[:, 0] <= full) and np.all(full <= enc[:, 1])
    assert np.all(enc[:, 2] <= 0.0) and np.all(0.0 <= enc[:, 3])


@CPU
@given(st.lists(st.integers(min_value=0, max_value=(1 << 40) - 1), min_size=1, max_size=200),
       st.integers(min_value=0, max_value=8))
def test_oracle_carry_rebuilds_the_integer(coeffs, extra):
    c = np.array(coeffs, dtype=np.int64)
    value = sum(int(v) << (8 * i) for i, v in enumerate(coeffs))
    nout = max(len(coeffs) + 6 + extra, (value.bit_length() + 7) // 8)
    out = oracle.carry(c, 8, nout)
    assert to_int(out) == value


@CPU
@given(operand, operand)
def test_long_multiplication_pin(a, b):
    assert np.array_equal(long_multiplication(a, b), int_product(a, b))


# ---- GPU -------------------------------------------------------------------

big_operand = st.integers(min_value=1, max_value=6000).flatmap(
    lambda n: st.binary(min_size=n, max_size=n)).map(lambda b: np.frombuffer(b, dtype=np.uint8).copy())
GPU = settings(max_examples=40, deadline=None, suppress_health_check=[HealthCheck.too_slow,
                                                                     HealthCheck.data_too_large])


@pytest.fixture(scope="module")
def plans():
    from paper_1006_0405_amd import binding
    p = {"rect": binding.Plan(6000, 6000), "exact": binding.Plan(6000, 6000, exact_fallback=True)}
    p["exact"].force_too_wide(True)  # every interval run refuses: the exact transform answers
    yield p
    for v in p.values():
        v.close()


@pytest.mark.gpu
@GPU
@given(a=big_operand, b=big_operand, ka=special, kb=special)
def test_gpu_product_properties(plans, a, b, ka, kb):
    from paper_1006_0405_amd import binding
    a, b = shaped(a, ka), shaped(b, kb)
    want = int_product(a, b)
    st_, out = plans["rect"].mul(a, b)
    ost = oracle.mul(a, b)[0] if len(a) * len(b) <= 1_000_000 else None
    if st_ == binding.SSA_OK:
        assert np.array_equal(out.cpu().numpy(), want)
    else:
        assert st_ == binding.SSA_ENCLOSURE_TOO_WIDE and not out.cpu().numpy().any()
    if ost is not None and ost == oracle.ST_OK:
        assert st_ == binding.SSA_OK  # the GPU's enclosures are narrower than the oracle's
    st_, out = plans["exact"].mul(a, b)
    assert st_ == binding.SSA_OK and np.array_equal(out.cpu().numpy(), want)
    st_, out = plans["rect"].mul_long(a, b)
    assert st_ == binding.SSA_OK and np.array_equal(out.cpu().numpy(), want)


@pytest.mark.gpu
@settings(max_examples=8, deadline=None, suppress_health_check=[HealthCheck.too_slow,
                                                                HealthCheck.data_too_large])
@given(st.lists(st.tuples(big_operand, big_operand), min_size=1, max_size=24))
def test_gpu_batch_properties(pairs):
    from paper_1006_0405_amd import binding
    A = [p[0] for p in pairs]
    B = [p[1] for p in pairs]
    plan = binding.Plan(6000, 6000)
    bt = binding.Batch(plan, A, B)
    st_ = bt.run().cpu().numpy()
    for i in range(len(A)):
        assert st_[i] == binding.SSA_OK
        assert np.array_equal(bt.OUT[i].cpu().numpy(), int_product(A[i], B[i])), i
    bt.close()
    plan.close()
