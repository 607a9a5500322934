"""A length class of more than 65,535 multi-pass products: the passes index
products by a grid dimension of at most 65,535, so such a class is launched in
chunks.  65,542 products of two 4,096-byte operands (N = 2^13, the shortest
multi-pass length) run through the eager launch path (ssa_batch_run_timed,
which launches the whole class at once, so the chunking takes effect) and
through the graph; every product must equal the integer product.  The
operands are one pair of device buffers shared by all products; the outputs
are rows of one buffer.  About 22 GB of device scratch.
"""
import ctypes

import pytest
import torch

from pins import int_product
from paper_1006_0405_amd import binding
from paper_1006_0405_amd.workloads import pair

pytestmark = pytest.mark.gpu

COUNT = 65535 + 7
NBYTES = 4096


def test_class_of_more_than_65535_products():
    print("%d products of %d x %d bytes in one length class" % (COUNT, NBYTES, NBYTES), flush=True)
    a, b = pair(65_000, NBYTES)
    want = torch.from_numpy(int_product(a, b).copy()).cuda()
    da = torch.from_numpy(a).cuda()
    db = torch.from_numpy(b).cuda()
    out = torch.zeros((COUNT, 2 * NBYTES), dtype=torch.uint8, device="cuda")
    status = torch.full((COUNT,), -1, dtype=torch.int32, device="cuda")
    plan = binding.Plan(NBYTES, NBYTES)
    L = binding.lib()
    vp = ctypes.c_void_p
    pa = (vp * COUNT)(*([da.data_ptr()] * COUNT))
    pb = (vp * COUNT)(*([db.data_ptr()] * COUNT))
    row = 2 * NBYTES
    po = (vp * COUNT)(*[out.data_ptr() + i * row for i in range(COUNT)])
    na = (ctypes.c_size_t * COUNT)(*([NBYTES] * COUNT))
    nb = (ctypes.c_size_t * COUNT)(*([NBYTES] * COUNT))
    h = vp()
    rc = L.ssa_batch_create(plan.handle, COUNT, ctypes.cast(pa, vp), ctypes.cast(na, vp),
                            ctypes.cast(pb, vp), ctypes.cast(nb, vp), ctypes.cast(po, vp),
                            ctypes.byref(h))
    assert rc == binding.SSA_OK, binding.STATUS_NAMES.get(rc, rc)
    try:
        for run in (L.ssa_batch_run_timed, L.ssa_batch_run):
            out.zero_()
            status.fill_(-1)
            assert run(h, status.data_ptr()) == binding.SSA_OK
            torch.cuda.synchronize()
            assert bool((status == binding.SSA_OK).all())
            good = (out == want).all(dim=1)
            assert bool(good.all()), int((~good).nonzero()[0])
    finally:
        L.ssa_batch_destroy(h)
        plan.close()
