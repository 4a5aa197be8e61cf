"""Leapfrog steps on the GPU (Sec. III.B.2: second-order leap-frog with a
full tree rebuild per step) against the oracle's FP64 kick-drift-kick with
oracle tree forces, both started from the same seeded initial conditions.

After every step the GPU's rebuilt tree must satisfy the octree's
invariants; the trajectory must agree with the oracle's to the FP32
rounding of the state.  (The oracle never sees a GPU result: the bit-exact
tree comparison is made on seeded inputs in the parity tests.)
"""
import numpy as np
import pytest

from gpu_util import cells_of, to_dev
from workloads import ics


def assert_tree_invariants(t, n):
    """Properties of any valid tree of n particles, checked on the GPU's."""
    keys = t.export("keys")
    assert np.all(keys[1:] >= keys[:-1])
    perm = t.export("perm").astype(np.int64)
    assert np.array_equal(np.sort(perm), np.arange(n))
    c = cells_of(t)
    leaf = c["nchild"] == 0
    assert c["count"][leaf].astype(np.int64).sum() == n
    internal = ~leaf
    ch = c["child0"][internal].astype(np.int64)
    # children of a cell partition its particles, the first child starts with it
    assert np.array_equal(c["begin"][ch], c["begin"][internal])
    assert t.export("group_count").astype(np.int64).sum() == n

pytestmark = pytest.mark.gpu


def _state(t):
    p, v = t.state()
    return p.cpu().numpy(), v.cpu().numpy()


def _oracle_kdk(oracle, pos, vel, mass, dt, steps, theta, eps):
    f = oracle.tree_force_fn(mass, theta, eps)
    return oracle.leapfrog(pos, vel, mass, dt, steps, f)


@pytest.mark.parametrize("pos_fp64", [False, True])
def test_steps_match_oracle(oracle, pos_fp64):
    import paper_1412_0659_amd as bh
    s = ics.disk_halo(10000, 40000, 51)
    theta, eps, dt, steps = 0.4, 0.005, 1e-3, 5
    t = bh.Tree(s.n, pos_fp64=pos_fp64)
    t.set_state(to_dev(s.pos), to_dev(s.vel), to_dev(s.mass))
    for k in range(steps):
        t.step(dt, theta, eps)
        assert_tree_invariants(t, s.n)
    p, v = _state(t)
    xo, vo = _oracle_kdk(oracle, s.pos, s.vel, s.mass, dt, steps, theta, eps)
    scale_x = np.abs(xo).max(1, keepdims=True) + 1.0
    ex = np.abs(p - xo) / scale_x
    ev = np.linalg.norm(v - vo, axis=1) / (np.linalg.norm(vo, axis=1) + 1e-3)
    print(f"pos_fp64={pos_fp64}: max pos err {ex.max():.2e}, vel err med {np.median(ev):.2e} "
          f"p99 {np.percentile(ev, 99):.2e}", flush=True)
    assert ex.max() <= 2e-6
    assert np.median(ev) <= 1e-5 and np.percentile(ev, 99) <= 1e-4
    t.close()


def test_energy_and_momentum():
    """Plummer sphere, 100 steps: energy error stays small (second-order
    scheme with a tree force) and the total momentum stays near zero."""
    import paper_1412_0659_amd as bh
    s = ics.plummer(4096, 52)
    theta, eps, dt = 0.5, 0.02, 2e-3
    m = s.mass.astype(np.float64)

    import torch
    every = torch.arange(s.n, dtype=torch.int64, device="cuda")

    def energy(t, v):
        # potential energy from the GPU's FP64 direct sum at the current state
        _, pot = t.direct(every, eps)
        t.sync()
        pot = pot.cpu().numpy()
        return 0.5 * (m * (v.astype(np.float64) ** 2).sum(1)).sum() + 0.5 * (m * pot).sum()

    t = bh.Tree(s.n)
    t.set_state(to_dev(s.pos), to_dev(s.vel), to_dev(s.mass))
    E0 = energy(t, s.vel)
    for _ in range(100):
        t.step(dt, theta, eps)
    p, v = _state(t)
    E1 = energy(t, v)
    mom = (m[:, None] * v).sum(0)
    print(f"dE/E {abs(E1 / E0 - 1):.2e}, |P| {np.linalg.norm(mom):.2e}", flush=True)
    assert abs(E1 / E0 - 1) <= 1e-3
    assert np.linalg.norm(mom) <= 1e-3 * (m * np.linalg.norm(v, axis=1)).sum()
    t.close()


def test_step_parameters_change():
    """A step with a different (theta, eps) recomputes the starting force."""
    import paper_1412_0659_amd as bh
    s = ics.plummer(2048, 53)
    a = bh.Tree(s.n)
    a.set_state(to_dev(s.pos), to_dev(s.vel), to_dev(s.mass))
    a.force(0.7, 0.05)
    a.step(1e-3, 0.4, 0.01)
    b = bh.Tree(s.n)
    b.set_state(to_dev(s.pos), to_dev(s.vel), to_dev(s.mass))
    b.step(1e-3, 0.4, 0.01)
    pa, va = _state(a)
    pb, vb = _state(b)
    assert np.array_equal(pa, pb) and np.array_equal(va, vb)
    a.close()
    b.close()
