"""FP16 far-field form (particle-cell terms in packed FP16 with FP32
accumulation, particle-particle terms in FP32) against the oracle.

The interaction lists are those of the FP32 walk, so the per-group counts
are bit-exact.  The forces carry FP16 rounding of order 2^-11 per
particle-cell term: against the FP64 oracle tree they must stay within
5e-4 median / 5e-3 99th percentile, and against the FP64 direct sum at
theta = 0.4 within 1e-3 median.
"""
import numpy as np
import pytest

from gpu_util import gpu_force, gpu_tree, rel_err
from workloads import ics

pytestmark = pytest.mark.gpu

MED16, P9916 = 5e-4, 5e-3


def _check(oracle, pos, mass, theta, eps, label):
    t = gpu_tree(pos, mass, far_fp16=True)
    acc, pot = gpu_force(t, theta, eps)
    ot = oracle.build_tree(pos, mass)
    oacc, opot, onpp, onpc = oracle.walk(ot, theta, eps)
    assert np.array_equal(t.export("group_npp").astype(np.int64), onpp)
    assert np.array_equal(t.export("group_npc").astype(np.int64), onpc)
    ea, ep = rel_err(acc, oacc), rel_err(pot, opot)
    print(f"{label}: acc med {np.median(ea):.2e} p99 {np.percentile(ea, 99):.2e}  "
          f"pot med {np.median(ep):.2e} p99 {np.percentile(ep, 99):.2e}", flush=True)
    assert np.all(np.isfinite(acc)) and np.all(np.isfinite(pot))
    assert np.median(ea) <= MED16 and np.percentile(ea, 99) <= P9916
    assert np.median(ep) <= MED16 and np.percentile(ep, 99) <= P9916
    t.close()
    return acc


@pytest.mark.parametrize("theta,eps", [(0.3, 0.005), (0.4, 0.005), (0.6, 0.005), (0.5, 0.0)])
def test_fp16_far_field_vs_oracle_tree(oracle, theta, eps):
    s = ics.disk_halo(20000, 80000, 41)
    _check(oracle, s.pos, s.mass, theta, eps, f"disk_halo_100k theta={theta} eps={eps}")


def test_fp16_far_field_plummer_and_clusters(oracle):
    s = ics.plummer(16384, 1)
    _check(oracle, s.pos, s.mass, 0.5, 0.01, "plummer_16k")
    rng = np.random.default_rng(9)
    pos = np.concatenate([rng.normal(size=(3000, 3)) * 1e-3, rng.uniform(-50, 50, (1500, 3)),
                          np.full((80, 3), 0.25)]).astype(np.float32)
    m = rng.uniform(0.5, 2.0, pos.shape[0]).astype(np.float32)
    _check(oracle, pos, m, 0.5, 1e-4, "clustered")


def test_fp16_far_field_vs_direct_sum(oracle):
    """The precision form's bar: median error <= 1e-3 against the FP64
    direct sum at theta = 0.4 (subsample of targets)."""
    s = ics.disk_halo(40000, 160000, 42)
    t = gpu_tree(s.pos, s.mass, far_fp16=True)
    acc, pot = gpu_force(t, 0.4, 0.005)
    t.close()
    t32 = gpu_tree(s.pos, s.mass)
    acc32, _ = gpu_force(t32, 0.4, 0.005)
    t32.close()
    sub = ics.subsample(s.n, 4096, 40)
    ad, _ = oracle.direct(s.pos, s.mass, 0.005, targets=sub)
    e16 = rel_err(acc[sub], ad)
    e32 = rel_err(acc32[sub], ad)
    print(f"vs direct: fp16 med {np.median(e16):.2e} p99 {np.percentile(e16, 99):.2e}; "
          f"fp32 med {np.median(e32):.2e} p99 {np.percentile(e32, 99):.2e}", flush=True)
    assert np.median(e16) <= 1e-3
    assert np.median(e16) <= 2.0 * np.median(e32) + 2e-4
