"""Writes tests/golden/oracle_samples.json: the CPU oracle's outcome on sampled
products of the batch workloads and on the two 1,000,000-byte products.

Calls only oracle/ (and the seeded input generators); nothing here comes from
the GPU library.  For every sampled product it stores the oracle's status, the
SHA-256 of its product bytes (all zeros when refused), its largest enclosure
radius and its half-integer count, for base-256 digits (the 4096-product batch
in FP64) and base-16 digits (the same batch re-split).  Run from the repository
root:  python tests/golden/make_oracle_samples.py  [--workers 6]
Takes several minutes: the two 2^22-point products dominate.
"""
import argparse
import hashlib
import json
import os
import sys
import time
from multiprocessing import get_context

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_samples.json")
SAMPLES = 256


def sample_indices(na, nb, count=SAMPLES):
    """`count` batch indices spread over every transform length class of the
    base-256 products: classes visited round-robin, each class's members taken
    in index order."""
    import oracle
    classes = {}
    for i in range(len(na)):
        classes.setdefault(oracle.fft_size(int(na[i]), int(nb[i]), 8), []).append(i)
    keys = sorted(classes)
    picked, r = [], 0
    while len(picked) < count:
        for k in keys:
            if r < len(classes[k]) and len(picked) < count:
                picked.append(classes[k][r])
        r += 1
    return sorted(picked)


def _job(args):
    kind, idx, bits = args
    import oracle
    from paper_1006_0405_amd.workloads import all_ff, batch, pair
    if kind == "batch":
        A, B = batch(seed=3)
        a, b = A[idx], B[idx]
    elif kind == "c5_random":
        a, b = pair(5, 1_000_000)
    else:
        a = b = all_ff(1_000_000)
    t0 = time.perf_counter()
    st, out, rad, half = oracle.mul(a, b, digit_bits=bits)
    return {"kind": kind, "index": idx, "digit_bits": bits, "na": len(a), "nb": len(b),
            "fft_length": oracle.fft_size(len(a), len(b), bits), "status": int(st),
            "sha256": hashlib.sha256(out.tobytes()).hexdigest(), "max_radius": rad,
            "half_int": int(half), "oracle_s": time.perf_counter() - t0}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=6)
    args = ap.parse_args()
    import oracle
    from paper_1006_0405_amd.workloads import batch_lengths
    oracle.lib()
    _, na, nb = batch_lengths(seed=3)
    idx = sample_indices(na, nb)
    jobs = [("c5_random", -1, 4), ("c5_all_ff", -1, 4)]
    jobs += [("batch", i, bits) for bits in (8, 4) for i in idx]
    with get_context("spawn").Pool(args.workers) as pool:
        res = []
        for r in pool.imap(_job, jobs):
            res.append(r)
            if r["kind"] != "batch" or len(res) % 64 == 0:
                print("%d/%d %s %.1f s" % (len(res), len(jobs), r["kind"], r["oracle_s"]), flush=True)
    doc = {
        "about": "CPU oracle (radix-2 FFT box over rectangular intervals, fesetround) on products "
                 "of the seeded workloads: 256 products of the 4096-product batch (seed 3, "
                 "log-uniform 64..16384 bytes) spread over every length class, in base 256 and "
                 "base 16; the 1,000,000 x 1,000,000-byte products in base 16 (random seed 5, "
                 "all 0xFF).  Written by tests/golden/make_oracle_samples.py.",
        "batch_indices": idx,
        "products": res,
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=0)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
