"""The entry point that allocates nothing (tree_force_static): its output
against the context path's (tree_build + tree_force with the same
parameters) on two calls in a row, the second with fewer particles, and at
the largest size it accepts."""
import numpy as np
import pytest

from gpu_util import device, to_dev
from workloads import ics

pytestmark = pytest.mark.gpu


def _static(pos, mass, theta, eps):
    import torch
    from paper_1412_0659_amd import binding as B
    n = mass.shape[0]
    acc = torch.full((n, 3), float("nan"), dtype=torch.float32, device="cuda")
    pot = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    B.tree_force_static(to_dev(pos), to_dev(mass), theta, eps, acc, pot, st)
    torch.cuda.synchronize()
    return acc.cpu().numpy(), pot.cpu().numpy(), int(st.cpu().item())


def _context(pos, mass, theta, eps):
    from paper_1412_0659_amd import Tree
    t = Tree(mass.shape[0])
    t.build(to_dev(pos), to_dev(mass))
    acc, pot = t.force(theta, eps)
    t.sync()
    out = acc.cpu().numpy(), pot.cpu().numpy()
    t.close()
    return out


def _cases():
    d = ics.disk_halo(10000, 50000, 61)
    yield "disk_halo_60k", d.pos, d.mass, 0.4, 0.005
    p = ics.plummer(5003, 62)  # a second, smaller call: the array keeps the first call's contents
    yield "plummer_5003", p.pos, p.mass, 0.5, 0.01
    m = ics.disk_halo(10923, 54613, 63)  # the largest n the entry point accepts
    yield "disk_halo_65536", m.pos, m.mass, 0.6, 0.002


def test_static_matches_context_path():
    device()
    from paper_1412_0659_amd import binding as B
    for name, pos, mass, theta, eps in _cases():
        print(f"case {name} n={mass.shape[0]} theta={theta} eps={eps}", flush=True)
        assert mass.shape[0] <= B.BH_STATIC_MAX_N
        a, p, st = _static(pos, mass, theta, eps)
        ra, rp = _context(pos, mass, theta, eps)
        assert st == 0
        # same kernels on the same inputs: bit-identical forces
        assert np.array_equal(a, ra) and np.array_equal(p, rp), name


def test_static_errors_and_status():
    import torch
    device()
    from paper_1412_0659_amd import binding as B
    s = ics.plummer(1000, 64)
    with pytest.raises(B.BhError) as e:
        big = np.zeros((B.BH_STATIC_MAX_N + 1, 3), np.float32)
        B.tree_force_static(to_dev(big), to_dev(np.ones(B.BH_STATIC_MAX_N + 1)), 0.5, 0.01)
    assert e.value.code == B.BH_ECAPACITY
    for theta, eps in [(0.0, 0.01), (1.5, 0.01), (0.5, -1.0)]:
        with pytest.raises(B.BhError) as e:
            B.tree_force_static(to_dev(s.pos), to_dev(s.mass), theta, eps)
        assert e.value.code == B.BH_EINVAL
    bad = s.mass.copy()
    bad[7] = 0.0
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    B.tree_force_static(to_dev(s.pos), to_dev(bad), 0.5, 0.01, None, None, st)
    torch.cuda.synchronize()
    assert int(st.cpu().item()) == 2  # mass <= 0
    # the next call starts from a clear status word
    a, p, st2 = _static(s.pos, s.mass, 0.5, 0.01)
    ra, rp = _context(s.pos, s.mass, 0.5, 0.01)
    assert st2 == 0 and np.array_equal(a, ra) and np.array_equal(p, rp)
