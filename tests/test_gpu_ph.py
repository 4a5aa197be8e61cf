"""The Peano-Hilbert curve (the paper's, Sec. III.B.1) on the GPU: keys,
sort order, cells, groups and FP64 moments bit-exact against the oracle's
Peano-Hilbert tree; the walk on it against the oracle; and the same forces
as the Morton tree, whose cells are the same."""
import numpy as np
import pytest

from gpu_util import assert_tree_equal, gpu_force, gpu_tree, rel_err
from workloads import ics

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n_disk,n_halo,seed", [(20000, 80000, 101), (300, 1200, 102)])
def test_ph_tree_bit_exact_and_walk(oracle, n_disk, n_halo, seed):
    s = ics.disk_halo(n_disk, n_halo, seed)
    t = gpu_tree(s.pos, s.mass, curve="ph")
    ot = oracle.build_tree(s.pos, s.mass, curve="ph")
    assert_tree_equal(t, ot)
    assert np.array_equal(t.export("mom_M"), ot.mom["M"])
    assert np.array_equal(t.export("mom_com"), ot.mom["com"])
    assert np.array_equal(t.export("mom_Q"), ot.mom["Q"])
    size = t.export("cell_size")
    assert np.array_equal(size[:, 1], ot.mom["deltaf"])
    acc, pot = gpu_force(t, 0.4, 0.005)
    oacc, opot, onpp, onpc = oracle.walk(ot, 0.4, 0.005)
    assert np.array_equal(t.export("group_npc").astype(np.int64), onpc)
    assert np.array_equal(t.export("group_npp").astype(np.int64), onpp)
    ea = rel_err(acc, oacc)
    print(f"  ph n={s.n}: acc med {np.median(ea):.2e} p99 {np.percentile(ea, 99):.2e}", flush=True)
    assert np.median(ea) <= 1e-5 and np.percentile(ea, 99) <= 1e-4
    # the Morton tree has the same cells: the same interaction totals, and
    # forces that differ only by summation order
    tm = gpu_tree(s.pos, s.mass)
    am, _ = gpu_force(tm, 0.4, 0.005)
    # (equal up to an opening decision that the FP64 summation order of a
    # cell's moments can tip after rounding to FP32)
    for k in ("n_pc", "n_pp"):
        assert abs(tm.stats()[k] - t.stats()[k]) <= 1e-6 * t.stats()[k]
    assert np.percentile(rel_err(acc, am), 99) <= 1e-5
    t.close()
    tm.close()
