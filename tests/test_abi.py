"""The C-ABI library loads and exports every symbol include/bh.h declares;
host-side argument checks that return before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "bh.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return re.findall(r"^\s*(?:int|int64_t|const char \*)\s*(\w+)\s*\(", src, flags=re.M)


def test_header_declares_the_boundary():
    names = set(_declared())
    for fn in ("tree_build", "tree_force", "leapfrog_step", "bh_create", "bh_destroy"):
        assert fn in names


def test_library_exports_every_declared_symbol():
    import paper_1412_0659_amd as bh
    L = bh.load()
    for name in _declared():
        assert hasattr(L, name), name
    assert set(_declared()) == set(bh.binding.SYMBOLS)


def test_host_argument_checks():
    import paper_1412_0659_amd as bh
    L = bh.load()
    assert L.bh_create(None, 10, None) == bh.binding.BH_EINVAL
    out = ctypes.c_void_p()
    assert L.bh_create(ctypes.byref(out), 0, None) == bh.binding.BH_EINVAL
    assert L.bh_create(ctypes.byref(out), -5, None) == bh.binding.BH_EINVAL
    for nleaf, ncrit, f16 in [(0, 64, 0), (16, 0, 0), (16, 65, 0), (65, 64, 0), (16, 64, 2)]:
        p = bh.binding.bh_params(nleaf, ncrit, f16, 0)
        assert L.bh_create(ctypes.byref(out), 100, ctypes.byref(p)) == bh.binding.BH_EINVAL
    for pg in (-1, 1, 65):
        p = bh.binding.bh_params(16, 64, 0, 0, 0, 0, pg)
        assert L.bh_create(ctypes.byref(out), 100, ctypes.byref(p)) == bh.binding.BH_EINVAL
    # too many particles for the 29-bit cell index of the walk stack
    assert L.bh_create(ctypes.byref(out), 1 << 28, None) == bh.binding.BH_EINVAL
    assert L.bh_destroy(None) == bh.binding.BH_EINVAL
    assert L.tree_build(None, None, None, 10, None) == bh.binding.BH_EINVAL
    assert L.tree_force(None, 0.5, 0.01, None, None, None) == bh.binding.BH_EINVAL
    assert L.leapfrog_step(None, 1e-3, 0.5, 0.01, None) == bh.binding.BH_EINVAL
    assert L.bh_sync(None, None) == bh.binding.BH_EINVAL
    assert L.tree_direct(None, None, 1, 0.01, None, None, None) == bh.binding.BH_EINVAL
    assert L.bh_diagnostics(None, None, None) == bh.binding.BH_EINVAL
    assert L.bh_export_keys(None, None, None, None) == bh.binding.BH_EINVAL
    assert L.bh_export_tree(None, None, None) == bh.binding.BH_EINVAL
    assert L.bh_strerror(bh.binding.BH_ESTATE) == b"call out of order"
    assert L.bh_last_error(None) == b""


def test_paper_flop_convention_reproduces_table2():
    """The 23 / 65 flop convention of Sec. VI.A reproduces the single-GPU
    Tflops of Table II from its own interaction counts and time."""
    from golden_io import key_values
    import bench
    t = key_values("paper_table2_1gpu.txt")
    n = t["n_particles"]
    flops = bench.paper_flops(n * t["pp_per_particle"], n * t["pc_per_particle"])
    assert abs(flops / t["gravity_s"] / 1e12 - t["gpu_tflops"]) < 0.01
    assert abs(flops / t["total_s"] / 1e12 - t["application_tflops"]) < 0.01
