"""Pins of the oracle's differentiation form: the hand-written adjoint of the
tree force with frozen decisions (Sec. VI.A Eq. (2) through the moments of
Sec. I.A / Eq. (1)), checked against central finite differences of the
frozen-decision force and, in the theta -> 0 limit, against torch.autograd
of a plain direct sum (FP64, CPU)."""
import numpy as np
import pytest

from workloads import ics


def _sorted_state(t):
    x = np.stack([t.x, t.y, t.z], 1).astype(np.float64)
    return x, t.m.astype(np.float64)


def test_replay_reproduces_walk(oracle):
    s = ics.disk_halo(500, 2000, 31)
    t = oracle.build_tree(s.pos, s.mass)
    d = oracle.record_decisions(t, 0.5)
    x, m = _sorted_state(t)
    a, p, *_ = oracle.replay(d, x, m, 0.01)
    acc, pot, npp, npc = oracle.walk(t, 0.5, 0.01)
    assert np.allclose(a, acc[t.perm], rtol=1e-12, atol=1e-15 * np.abs(acc).max())
    assert np.allclose(p, pot[t.perm], rtol=1e-12)
    assert np.array_equal(np.diff(d.pc_off), npc)


@pytest.mark.parametrize("theta,eps", [(0.4, 0.01), (0.7, 0.0), (0.3, 0.05)])
def test_vjp_matches_finite_differences(oracle, theta, eps):
    s = ics.disk_halo(400, 1600, 32)
    t = oracle.build_tree(s.pos, s.mass)
    d = oracle.record_decisions(t, theta)
    x, m = _sorted_state(t)
    rng = np.random.default_rng(5)
    u = rng.normal(size=x.shape)
    gx, gm = oracle.replay_vjp(d, x, m, eps, u)
    scale = np.abs(x).max()
    for _ in range(16):
        dx = rng.normal(size=x.shape)
        dm = rng.normal(size=m.shape) * m
        h = 1e-6 * scale
        fp = oracle.replay(d, x + h * dx / scale, m + h * dm / scale, eps)[0]
        fm = oracle.replay(d, x - h * dx / scale, m - h * dm / scale, eps)[0]
        fd = (u * (fp - fm)).sum() / (2 * h) * scale
        an = (gx * dx).sum() + (gm * dm).sum()
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-12, (fd, an)


def test_vjp_direct_limit_matches_torch_autograd(oracle):
    torch = pytest.importorskip("torch")
    s = ics.plummer(300, 33)
    t = oracle.build_tree(s.pos, s.mass)
    d = oracle.record_decisions(t, 1e-6)
    assert d.pc_off[-1] == 0
    x, m = _sorted_state(t)
    eps = 0.02
    rng = np.random.default_rng(6)
    u = rng.normal(size=x.shape)
    gx, gm = oracle.replay_vjp(d, x, m, eps, u)
    X = torch.tensor(x, requires_grad=True)
    Mt = torch.tensor(m, requires_grad=True)
    r = X[None, :, :] - X[:, None, :]            # r_ij = x_j - x_i
    r2 = (r * r).sum(-1) + eps * eps
    w = Mt[None, :] * r2 ** -1.5
    w = w * (1.0 - torch.eye(len(m), dtype=torch.float64))
    acc = (w[:, :, None] * r).sum(1)
    (acc * torch.tensor(u)).sum().backward()
    assert np.allclose(gx, X.grad.numpy(), rtol=1e-10, atol=1e-12 * np.abs(gx).max())
    assert np.allclose(gm, Mt.grad.numpy(), rtol=1e-10, atol=1e-12 * np.abs(gm).max())
