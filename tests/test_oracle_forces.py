"""Pins of the oracle's force arithmetic: direct summation and the
particle-cell expansion of Sec. VI.A Eq. (1)-(2), with Plummer softening.

Pinned against closed forms (two-body, the Plummer sphere), an invariant
(Newton's third law), the identity a = -grad(phi), and the convergence order
of the quadrupole expansion against an exact direct sum.
"""
import numpy as np

from golden_io import key_values
from workloads import ics


def test_two_body_closed_form(oracle):
    eps = 0.3
    pos = np.array([[0.0, 0.0, 0.0], [1.2, -0.5, 2.0]])
    m = np.array([0.7, 1.9])
    acc, pot = oracle.direct(pos, m, eps)
    r = pos[1] - pos[0]
    s2 = r @ r + eps * eps
    assert np.allclose(acc[0], m[1] * r / s2 ** 1.5, rtol=1e-15, atol=0)
    assert np.allclose(acc[1], -m[0] * r / s2 ** 1.5, rtol=1e-15, atol=0)
    assert np.isclose(pot[0], -m[1] / np.sqrt(s2), rtol=1e-15)
    assert np.isclose(pot[1], -m[0] / np.sqrt(s2), rtol=1e-15)
    # a single particle feels nothing
    a1, p1 = oracle.direct(pos[:1], m[:1], eps)
    assert np.all(a1 == 0) and p1[0] == 0


def test_newton_third_law(oracle):
    rng = np.random.default_rng(1)
    pos = rng.normal(size=(2000, 3))
    m = rng.uniform(0.1, 2.0, 2000)
    acc, _ = oracle.direct(pos, m, 0.05)
    mom = (m[:, None] * acc).sum(0)
    assert np.linalg.norm(mom) <= 1e-13 * (m * np.linalg.norm(acc, axis=1)).sum()


def test_plummer_closed_form(oracle):
    """W = -3 pi / 32, virial equilibrium, and the radial acceleration
    -r / (1 + r^2)^(3/2) averaged in 32 equal-count shells over 4 samples."""
    W_ref = key_values("plummer_closed_form.txt")["W"]
    Ws, rs, ars = [], [], []
    for seed in (1, 2, 3, 4):
        s = ics.plummer(16384, seed)
        acc, pot = oracle.direct(s.pos, s.mass, 1e-3)
        m = s.mass.astype(np.float64)
        W = 0.5 * (m * pot).sum()
        Ws.append(W)
        assert abs(W / W_ref - 1) < 0.03
        K = 0.5 * (m * (s.vel.astype(np.float64) ** 2).sum(1)).sum()
        assert abs((2 * K + W) / W) < 0.05
        x = s.pos.astype(np.float64)
        r = np.linalg.norm(x, axis=1)
        rs.append(r)
        ars.append((acc * x).sum(1) / r)
    assert abs(np.mean(Ws) / W_ref - 1) < 0.02
    r = np.concatenate(rs)
    ar = np.concatenate(ars)
    order = np.argsort(r)
    for k, sh in enumerate(np.array_split(order, 32)):
        if k == 0:
            continue
        want = np.mean(-r[sh] / (1 + r[sh] ** 2) ** 1.5)
        assert abs(ar[sh].mean() / want - 1) < 0.03, k


def _cluster(rng, n=64, s=1.0):
    pos = rng.normal(size=(n, 3)) * s * np.array([1.0, 0.6, 0.3])
    m = rng.uniform(0.5, 1.5, n)
    return pos, m


def test_expansion_is_gradient_of_potential(oracle):
    """Eq. (2) must be minus the gradient of Eq. (1) for any symmetric Q."""
    rng = np.random.default_rng(3)
    for eps in (0.0, 0.4):
        comc = rng.normal(size=3)
        A = rng.normal(size=(3, 3))
        Qm = A @ A.T
        q6 = np.array([Qm[0, 0], Qm[1, 1], Qm[2, 2], Qm[0, 1], Qm[0, 2], Qm[1, 2]])
        tgt = rng.normal(size=(20, 3)) * 3 + 4
        acc, _ = oracle.expansion(tgt, 1.3, comc, q6, eps)
        h = 1e-5
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            _, pp = oracle.expansion(tgt + e, 1.3, comc, q6, eps)
            _, pm = oracle.expansion(tgt - e, 1.3, comc, q6, eps)
            fd = -(pp - pm) / (2 * h)
            assert np.allclose(acc[:, a], fd, rtol=1e-7, atol=1e-9 * np.abs(acc).max())


def test_expansion_converges_at_third_order(oracle):
    """Error of the monopole+quadrupole expansion of a cluster (moments from
    the oracle's upward pass) against the exact direct sum falls like
    (s/d)^3; a wrong quadrupole sign or convention leaves (s/d)^2."""
    rng = np.random.default_rng(4)
    pos, m = _cluster(rng)
    t = oracle.build_tree(pos.astype(np.float32), m.astype(np.float32), nleaf=1000)
    assert t.cells["ncell"] == 1
    mc, comc, q6 = t.mom["M"][0], t.mom["com"][0], t.mom["Q"][0]
    xs = np.stack([t.x, t.y, t.z], 1).astype(np.float64)
    ms = t.m.astype(np.float64)
    dirn = rng.normal(size=(16, 3))
    dirn /= np.linalg.norm(dirn, axis=1, keepdims=True)
    errs, errs_mono = [], []
    for d in (8.0, 16.0, 32.0):
        tgt = comc + d * dirn
        allpos = np.concatenate([xs, tgt])
        allm = np.concatenate([ms, np.zeros(len(tgt))])
        ad, pd = oracle.direct(allpos, allm, 0.0, targets=np.arange(len(xs), len(allpos)))
        ae, pe = oracle.expansion(tgt, mc, comc, q6, 0.0)
        am, pm = oracle.expansion(tgt, mc, comc, np.zeros(6), 0.0)
        errs.append(np.max(np.linalg.norm(ae - ad, axis=1) / np.linalg.norm(ad, axis=1)))
        errs_mono.append(np.max(np.linalg.norm(am - ad, axis=1) / np.linalg.norm(ad, axis=1)))
    for k in range(2):
        assert 6.0 <= errs[k] / errs[k + 1] <= 10.0, errs
        assert 3.0 <= errs_mono[k] / errs_mono[k + 1] <= 5.0, errs_mono
    assert errs[0] < 0.2 * errs_mono[0]
