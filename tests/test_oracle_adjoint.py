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


# --- K-step leapfrog with frozen decisions ----------------------------------

def _trajectory(oracle, s, theta, eps, dt, steps):
    """FP32 positions of a tree-code KDK run (the trees the decisions come from)."""
    m = s.mass.astype(np.float64)
    f = oracle.tree_force_fn(s.mass, theta, eps)
    x, v = s.pos.astype(np.float64), s.vel.astype(np.float64)
    poss = [s.pos.copy()]
    for _ in range(steps):
        x, v = oracle.leapfrog(x, v, m, dt, 1, f)
        poss.append(x.astype(np.float32))
    return poss


def test_frozen_leapfrog_direct_limit_is_plain_leapfrog(oracle):
    """With every decision a p-p pair the frozen K-step map is the FP64 KDK
    leapfrog of Sec. III.B.2 on the direct sum."""
    s = ics.plummer(256, 41)
    m = s.mass.astype(np.float64)
    eps, dt, K = 0.02, 2e-3, 5
    poss = _trajectory(oracle, s, 1e-6, eps, dt, K)
    decs = oracle.trajectory_decisions(poss, s.mass, 1e-6)
    assert all(d.pc_off[-1] == 0 for d in decs)
    xK, vK, _ = oracle.leapfrog_frozen(s.pos, s.vel, m, dt, decs, eps)
    xr, vr = oracle.leapfrog(s.pos, s.vel, m, dt, K, oracle.direct_force_fn(m, eps))
    assert np.allclose(xK, xr, rtol=1e-12, atol=1e-14)
    assert np.allclose(vK, vr, rtol=1e-11, atol=1e-13 * np.abs(vr).max())


def test_frozen_leapfrog_vjp_matches_finite_differences(oracle):
    s = ics.disk_halo(120, 480, 42)
    m = s.mass.astype(np.float64)
    theta, eps, dt, K = 0.5, 0.01, 1e-3, 5
    decs = oracle.trajectory_decisions(_trajectory(oracle, s, theta, eps, dt, K), s.mass, theta)
    rng = np.random.default_rng(7)
    wx, wv = rng.normal(size=(600, 3)), rng.normal(size=(600, 3))
    gx, gv, gm = oracle.leapfrog_frozen_vjp(s.pos, s.vel, m, dt, decs, eps, wx, wv)

    def L(a, b, c):
        xk, vk, _ = oracle.leapfrog_frozen(a, b, c, dt, decs, eps)
        return (wx * xk).sum() + (wv * vk).sum()

    for _ in range(16):
        dx, dv = rng.normal(size=(600, 3)), rng.normal(size=(600, 3))
        dm = rng.normal(size=600) * m
        h = 1e-6
        fd = (L(s.pos + h * dx, s.vel + h * dv, m + h * dm)
              - L(s.pos - h * dx, s.vel - h * dv, m - h * dm)) / (2 * h)
        an = (gx * dx).sum() + (gv * dv).sum() + (gm * dm).sum()
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-9, (fd, an)


def test_frozen_leapfrog_vjp_direct_limit_matches_torch_autograd(oracle):
    """theta -> 0: the reverse sweep equals torch.autograd through K KDK
    steps of a plain FP64 direct sum."""
    torch = pytest.importorskip("torch")
    s = ics.plummer(160, 43)
    m = s.mass.astype(np.float64)
    eps, dt, K = 0.02, 2e-3, 4
    decs = oracle.trajectory_decisions(_trajectory(oracle, s, 1e-6, eps, dt, K), s.mass, 1e-6)
    rng = np.random.default_rng(8)
    wx, wv = rng.normal(size=(160, 3)), rng.normal(size=(160, 3))
    gx, gv, gm = oracle.leapfrog_frozen_vjp(s.pos, s.vel, m, dt, decs, eps, wx, wv)

    X0 = torch.tensor(s.pos.astype(np.float64), requires_grad=True)
    V0 = torch.tensor(s.vel.astype(np.float64), requires_grad=True)
    Mt = torch.tensor(m, requires_grad=True)
    off = 1.0 - torch.eye(160, dtype=torch.float64)

    def acc(X):
        r = X[None, :, :] - X[:, None, :]
        w = Mt[None, :] * ((r * r).sum(-1) + eps * eps) ** -1.5 * off
        return (w[:, :, None] * r).sum(1)

    X, V = X0, V0
    a = acc(X)
    for _ in range(K):
        V = V + 0.5 * dt * a
        X = X + dt * V
        a = acc(X)
        V = V + 0.5 * dt * a
    ((X * torch.tensor(wx)).sum() + (V * torch.tensor(wv)).sum()).backward()
    for mine, ref in ((gx, X0.grad), (gv, V0.grad), (gm, Mt.grad)):
        ref = ref.numpy()
        assert np.allclose(mine, ref, rtol=1e-9, atol=1e-11 * np.abs(ref).max())


# --- cloud-in-cell surface density --------------------------------------------

GRID = (0.2, 4.0, 8, 8)


def _area(grid, i):
    r0, r1, nr, nphi = grid
    dr = (r1 - r0) / nr
    a, b = r0 + i * dr, r0 + (i + 1) * dr
    return 0.5 * (2 * np.pi / nphi) * (b * b - a * a)


def _at(R, phi, z=0.0):
    return np.array([[R * np.cos(phi), R * np.sin(phi), z]])


def test_cic_particle_at_a_cell_centre_fills_one_cell(oracle):
    r0, r1, nr, nphi = GRID
    dr, dphi = (r1 - r0) / nr, 2 * np.pi / nphi
    for i, j in [(0, 0), (3, 5), (7, 7)]:
        sig = oracle.cic_density(_at(r0 + (i + 0.5) * dr, (j + 0.5) * dphi, 0.3), [2.5], None,
                                 GRID)
        ref = np.zeros((nr, nphi))
        ref[i, j] = 2.5 / _area(GRID, i)
        assert np.allclose(sig, ref, rtol=1e-12, atol=1e-12)


def test_cic_splits_across_the_periodic_phi_seam_and_in_radius(oracle):
    r0, r1, nr, nphi = GRID
    dr = (r1 - r0) / nr
    sig = oracle.cic_density(_at(r0 + 2.5 * dr, 0.0), [1.0], None, GRID)
    assert np.isclose(sig[2, 0] * _area(GRID, 2), 0.5)
    assert np.isclose(sig[2, nphi - 1] * _area(GRID, 2), 0.5)
    assert np.isclose(sig.sum(), 1.0 / _area(GRID, 2))
    sig = oracle.cic_density(_at(r0 + 3.25 * dr, (4 + 0.5) * 2 * np.pi / nphi), [1.0], None,
                             GRID)
    assert np.isclose(sig[2, 4] * _area(GRID, 2), 0.25)
    assert np.isclose(sig[3, 4] * _area(GRID, 3), 0.75)


def test_cic_conserves_mass_inside_and_drops_outside(oracle):
    rng = np.random.default_rng(9)
    r0, r1, nr, nphi = GRID
    dr = (r1 - r0) / nr
    R = rng.uniform(r0 + 0.5 * dr, r1 - 0.5 * dr, 500)
    phi = rng.uniform(0, 2 * np.pi, 500)
    pos = np.stack([R * np.cos(phi), R * np.sin(phi), rng.normal(size=500)], 1)
    m = rng.uniform(0.5, 1.5, 500)
    sig = oracle.cic_density(pos, m, None, GRID)
    areas = np.array([_area(GRID, i) for i in range(nr)])
    assert np.isclose((sig * areas[:, None]).sum(), m.sum(), rtol=1e-12)
    far = np.array([[0.0, r1 + dr, 0.0], [0.01, 0.0, 0.0]])
    assert not oracle.cic_density(far, [1.0, 1.0], None, GRID).any()
    sel = np.zeros(500, bool)
    sel[::3] = True
    assert np.allclose(oracle.cic_density(pos, m, sel, GRID),
                       oracle.cic_density(pos[sel], m[sel], None, GRID))


def test_cic_vjp_matches_finite_differences(oracle):
    s = ics.disk_halo(300, 300, 44)
    rng = np.random.default_rng(10)
    g = rng.normal(size=GRID[2:])
    sel = s.is_disk
    m = s.mass.astype(np.float64)
    gp, gm = oracle.cic_density_vjp(s.pos, m, sel, GRID, g)
    assert not gp[~sel].any() and not gm[~sel].any()
    assert not gp[:, 2].any()
    L = lambda p, mm: (g * oracle.cic_density(p, mm, sel, GRID)).sum()
    for _ in range(8):
        dp = rng.normal(size=(600, 3))
        dm = rng.normal(size=600) * m
        h = 1e-7
        fd = (L(s.pos + h * dp, m + h * dm) - L(s.pos - h * dp, m - h * dm)) / (2 * h)
        an = (gp * dp).sum() + (gm * dm).sum()
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-10, (fd, an)


def test_surface_density_loss_chain_matches_finite_differences(oracle):
    """The whole differentiation workload on the oracle: K frozen KDK steps,
    cloud-in-cell density of the disk, squared error against a target from
    perturbed initial conditions; reverse sweep vs central differences."""
    s = ics.disk_halo_scaled(1024, 45)
    m = s.mass.astype(np.float64)
    theta, eps, dt, K = 0.4, 0.005, 1e-3, 6
    tgt = ics.perturbed(s, 46)
    xt, _ = oracle.leapfrog(tgt.pos, tgt.vel, m, dt, K, oracle.tree_force_fn(s.mass, theta, eps))
    target = oracle.cic_density(xt, m, s.is_disk, GRID)
    poss = oracle.kdk_positions(s.pos, s.vel, s.mass, dt, K,
                                oracle.tree_force_fn(s.mass, theta, eps))
    decs = oracle.trajectory_decisions(poss, s.mass, theta)
    x0, v0 = s.pos.astype(np.float64), s.vel.astype(np.float64)

    def loss(x, v, mm):
        xK, _, _ = oracle.leapfrog_frozen(x, v, mm, dt, decs, eps)
        return ((oracle.cic_density(xK, mm, s.is_disk, GRID) - target) ** 2).sum()

    xK, _, _ = oracle.leapfrog_frozen(x0, v0, m, dt, decs, eps)
    gsig = 2 * (oracle.cic_density(xK, m, s.is_disk, GRID) - target)
    gxK, gmK = oracle.cic_density_vjp(xK, m, s.is_disk, GRID, gsig)
    gx, gv, gm = oracle.leapfrog_frozen_vjp(x0, v0, m, dt, decs, eps, gxK, np.zeros_like(gxK))
    gm = gm + gmK
    rng = np.random.default_rng(11)
    for _ in range(4):
        dx, dv, dm = rng.normal(size=x0.shape), rng.normal(size=v0.shape), rng.normal(size=1024) * m
        h = 1e-6
        fd = (loss(x0 + h * dx, v0 + h * dv, m + h * dm)
              - loss(x0 - h * dx, v0 - h * dv, m - h * dm)) / (2 * h)
        an = (gx * dx).sum() + (gv * dv).sum() + (gm * dm).sum()
        assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)


def test_kdk_positions_are_the_leapfrog_trajectory(oracle):
    s = ics.plummer(128, 47)
    m = s.mass.astype(np.float64)
    f = oracle.direct_force_fn(m, 0.02)
    poss = oracle.kdk_positions(s.pos, s.vel, s.mass, 1e-3, 3, f)
    assert len(poss) == 4 and np.array_equal(poss[0], s.pos)
    x3, _ = oracle.leapfrog(s.pos, s.vel, m, 1e-3, 3, f)
    assert np.array_equal(poss[3], x3.astype(np.float32))
