"""ssa_mul_noalloc against ssa_mul: the same products, bit for bit, with the
scratch in the library's static device array instead of a plan's allocations.

Two calls in a row share that array; the second, smaller one must not see the
first one's contents (statistics and carry state start from zero), and an
all-0xFF product, whose every carry ripples, follows a random one.
"""
import numpy as np
import pytest
import torch

from pins import int_product
from paper_1006_0405_amd import binding
from paper_1006_0405_amd.workloads import all_ff, pair

pytestmark = pytest.mark.gpu


def _noalloc(a, b):
    da = torch.from_numpy(a).cuda()
    db = torch.from_numpy(b).cuda()
    out = torch.full((len(a) + len(b),), 0xAB, dtype=torch.uint8, device="cuda")
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    binding.mul_noalloc(da, db, out, st)
    torch.cuda.synchronize()
    return int(st.cpu()[0]), out.cpu().numpy()


def _with_plan(a, b):
    plan = binding.Plan(len(a), len(b))
    try:
        st, out = plan.mul(a, b)
        return st, out.cpu().numpy()
    finally:
        plan.close()


CASES = [
    ("75000x75000 random, then 1024x1024 random", [pair(2, 75000), pair(1, 1024)]),
    ("6000x5000 random, then 300x17 random", [pair(3, 6000, 5000), pair(4, 300, 17)]),
    ("75000x75000 random, then 75000x75000 all-0xFF, then 40000x9 all-0xFF",
     [pair(5, 75000), (all_ff(75000), all_ff(75000)), (all_ff(40000), all_ff(9))]),
]


@pytest.mark.parametrize("name,ops", CASES, ids=[c[0] for c in CASES])
def test_noalloc_matches_ssa_mul(name, ops):
    print("ssa_mul_noalloc:", name, flush=True)
    for a, b in ops:
        st, out = _noalloc(a, b)
        pst, pout = _with_plan(a, b)
        assert st == pst == binding.SSA_OK, (len(a), len(b), st, pst)
        assert np.array_equal(out, pout), (len(a), len(b))
        assert np.array_equal(out, int_product(a, b)), (len(a), len(b))


def test_noalloc_rejects_sizes_beyond_its_maximum():
    a = torch.ones(1 << 17, dtype=torch.uint8, device="cuda")
    b = torch.ones((1 << 17) + 2, dtype=torch.uint8, device="cuda")
    out = torch.empty(a.numel() + b.numel(), dtype=torch.uint8, device="cuda")
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    with pytest.raises(binding.SsaError, match="INVALID_ARGUMENT"):
        binding.mul_noalloc(a, b, out, st)  # 2^18 + 1 coefficients
    b = b[:(1 << 17) + 1]
    out = out[:a.numel() + b.numel()]
    binding.mul_noalloc(a, b, out, st)  # exactly 2^18 coefficients
    torch.cuda.synchronize()
    want = int_product(np.ones(1 << 17, np.uint8), np.ones((1 << 17) + 1, np.uint8))
    assert int(st.cpu()[0]) == binding.SSA_OK
    assert np.array_equal(out.cpu().numpy(), want)
