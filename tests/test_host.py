"""Host-side checks that need no GPU: the C ABI library loads and exports
every entry point its header declares, the host-only size logic, and the
seeded workload generators."""
import ctypes
import os
import re

import numpy as np

from paper_1006_0405_amd import binding, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_entry_points():
    text = open(os.path.join(ROOT, "include", "ssa.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ssa_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_entry_point():
    declared = _declared_entry_points()
    assert len(declared) >= 10
    lib = ctypes.CDLL(binding.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(binding.EXPORTS) == declared


def test_fft_size_follows_the_fast_convolution_box():
    # N = 2^ceil(log2(L)), L = digits(a) + digits(b) - 1, padded to at least 512
    assert binding.fft_size(1024, 1024) == 2048
    assert binding.fft_size(75000, 75000) == 1 << 18
    assert binding.fft_size(1_000_000, 1_000_000, 4) == 1 << 22
    assert binding.fft_size(1, 1) == 512
    assert binding.fft_size(257, 1) == 512
    assert binding.fft_size(258, 256) == 1024
    assert binding.fft_size(128, 128, 4) == 512
    assert binding.fft_size(0, 5) == 0
    assert binding.fft_size(5, 5, 7) == 0


def test_workloads_are_seeded_and_shaped():
    a1, b1 = workloads.pair(1, 1024)
    a2, b2 = workloads.pair(1, 1024)
    assert np.array_equal(a1, a2) and np.array_equal(b1, b2)
    assert a1[-1] != 0 and b1[-1] != 0 and not np.array_equal(a1, b1)
    _, na, nb = workloads.batch_lengths(3)
    assert len(na) == 4096 and na.min() >= 64 and nb.max() <= 16384
    # log-uniform: about half the lengths below the geometric mean 1024
    assert 0.4 < np.mean(na < 1024) < 0.6


def _struct_fields(name):
    """Field names of `typedef struct { ... } name;` in the header, in order."""
    text = open(os.path.join(ROOT, "include", "ssa.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    m = re.search(r"typedef struct \{([^{}]*)\}\s*" + name + r"\s*;", text)
    assert m, name
    return [re.findall(r"(\w+)\s*$", decl.strip())[0] for decl in m.group(1).split(";") if decl.strip()]


def test_binding_structures_mirror_the_header():
    # the ctypes structures are passed by pointer through the C ABI: same fields, same order
    for cname, cls in (("ssa_plan_opts", binding.PlanOpts), ("ssa_launch_config", binding.LaunchConfig),
                       ("ssa_stats", binding.Stats)):
        assert [f[0] for f in cls._fields_] == _struct_fields(cname), cname
