"""Build libssa.so (the HIP library behind include/ssa.h) for gfx950.

Every HIP source is compiled with hipcc for gfx950 only.  Packed FP32
instructions are disabled (-packed-fp32-ops off).  After linking, the device
assembly of every source is generated and checked: the only writes of the
MODE register must be the library's own switch to FP64 round-toward-+inf
(the interval arithmetic depends on nothing else changing it).
"""
import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libssa.so")
SOURCES = ["api.hip", "kernels.hip", "twiddle.hip", "noalloc.hip", "ntt.hip", "lm.hip"]
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-fno-fast-math", "-ffp-contract=on", "-Wall"]

OWN_MODE_WRITE = "s_setreg_imm32_b32 hwreg(HW_REG_MODE, 2, 2), 1"


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("command failed: " + " ".join(cmd))
    return r


def _isa_of(src, verbose):
    asm = os.path.join("/tmp", f"ssa_isa_{os.getpid()}_{src}.s")
    _run(["hipcc", *COMMON, "--offload-device-only", "-S", os.path.join(CSRC, src), "-o", asm],
         verbose)
    text = open(asm).read()
    os.remove(asm)
    return text


def check_isa(verbose=False):
    """Generate device assembly and verify the MODE-register discipline."""
    bad = []
    with ThreadPoolExecutor(len(SOURCES)) as ex:
        texts = list(ex.map(lambda s: _isa_of(s, verbose), SOURCES))
    for src, text in zip(SOURCES, texts):
        for line in text.splitlines():
            t = line.strip()
            if re.match(r"s_setreg|s_round_mode|s_denorm_mode", t) and t != OWN_MODE_WRITE:
                bad.append(f"{src}: {t}")
    if bad:
        raise RuntimeError("unexpected MODE register writes in device code:\n" + "\n".join(bad))


def build(verbose=False, check=True):
    objs = [os.path.join("/tmp", f"ssa_{os.getpid()}_{src}.o") for src in SOURCES]
    with ThreadPoolExecutor(len(SOURCES)) as ex:
        list(ex.map(lambda so: _run(["hipcc", *COMMON, "-c", os.path.join(CSRC, so[0]), "-o", so[1]],
                                    verbose), zip(SOURCES, objs)))
    tmp = LIB + ".tmp"
    _run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp], verbose)
    for o in objs:
        os.remove(o)
    os.replace(tmp, LIB)
    if check:
        check_isa(verbose)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
