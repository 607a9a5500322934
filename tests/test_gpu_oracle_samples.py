"""Batch and 2^22-point products against the oracle's stored outcomes.

tests/golden/oracle_samples.json holds what the CPU oracle (and only the
oracle: tests/golden/make_oracle_samples.py calls nothing else) computes for
256 products of the 4096-product batch, spread over every length class, in
base 256 and in base 16, and for the two 1,000,000-byte products in base 16:
status, SHA-256 of the product bytes, largest radius and half-integer count.

The GPU runs the whole batch (FP64 rectangles; base 16 also with the FP32
first attempt) and the single products.  Where the oracle certifies, the GPU
must certify and return the same bytes.  Where the oracle refuses, the GPU may
certify (its enclosures are narrower) and must then return the integer
product.  The radii are printed side by side, per length class.
"""
import hashlib
import json
import os

import numpy as np
import pytest

from pins import int_product
from paper_1006_0405_amd import binding
from paper_1006_0405_amd.workloads import all_ff, batch, pair

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_samples.json")


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


def _check(gpu_status, gpu_bytes, gpu_radius, ref, a, b, rows):
    if ref["status"] == binding.SSA_OK:
        assert gpu_status == binding.SSA_OK, ref
        assert hashlib.sha256(gpu_bytes.tobytes()).hexdigest() == ref["sha256"], ref
    else:
        assert ref["status"] == binding.SSA_ENCLOSURE_TOO_WIDE, ref
        assert gpu_status in (binding.SSA_OK, binding.SSA_ENCLOSURE_TOO_WIDE)
        if gpu_status == binding.SSA_OK:
            assert np.array_equal(gpu_bytes, int_product(a, b)), ref
        else:
            assert not gpu_bytes.any()
    rows.setdefault(ref["fft_length"], []).append((gpu_radius, ref["max_radius"], ref["status"],
                                                   gpu_status))


def _report(rows, what):
    for n in sorted(rows):
        r = rows[n]
        print("%s N=%6d: %3d products, max radius GPU %.3e, oracle %.3e; oracle refused %d, "
              "GPU refused %d" % (what, n, len(r), max(x[0] for x in r), max(x[1] for x in r),
                                  sum(x[2] != 0 for x in r), sum(x[3] != 0 for x in r)))


@pytest.mark.parametrize("digit_bits,precision", [(8, "fp64"), (4, "fp64"), (4, "fp32_fallback")],
                         ids=["base256_fp64", "base16_fp64", "base16_fp32_fallback"])
def test_batch_samples_vs_oracle(digit_bits, precision):
    g = _golden()
    refs = {p["index"]: p for p in g["products"] if p["kind"] == "batch" and p["digit_bits"] == digit_bits}
    assert len(refs) == 256
    A, B = batch(seed=3)
    plan = binding.Plan(16384, 16384, digit_bits=digit_bits, precision=precision)
    bt = binding.Batch(plan, A, B)
    status = bt.run().cpu().numpy()
    stats = bt.stats()
    rows = {}
    for i, ref in sorted(refs.items()):
        assert (ref["na"], ref["nb"]) == (len(A[i]), len(B[i]))
        _check(int(status[i]), bt.OUT[i].cpu().numpy(), stats[i]["max_radius"], ref, A[i], B[i],
               rows)
    _report(rows, "base %d %s" % (1 << digit_bits, precision))
    bt.close()
    plan.close()


@pytest.mark.parametrize("kind", ["c5_random", "c5_all_ff"])
def test_config5_vs_oracle(kind):
    """1,000,000 x 1,000,000 bytes in base 16 (N = 2^22) against the oracle's
    stored outcome; the radius quoted beside the oracle's comes from here."""
    ref = [p for p in _golden()["products"] if p["kind"] == kind][0]
    a, b = pair(5, 1_000_000) if kind == "c5_random" else (all_ff(1_000_000), all_ff(1_000_000))
    plan = binding.Plan(len(a), len(b), digit_bits=4)
    st, out = plan.mul(a, b)
    s = plan.stats()
    rows = {}
    _check(st, out.cpu().numpy(), s["max_radius"], ref, a, b, rows)
    assert s["log_n"] == 22 and ref["fft_length"] == 1 << 22
    print("%s: status GPU %d oracle %d; max radius GPU %.4g, oracle %.4g; half-integers GPU %d, "
          "oracle %d" % (kind, st, ref["status"], s["max_radius"], ref["max_radius"], s["half_int"],
                         ref["half_int"]))
    plan.close()
