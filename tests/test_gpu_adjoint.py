"""Parity of the differentiation form on the GPU against the oracle.

* tree_force_vjp against the oracle's hand-written adjoint of the
  frozen-decision force (same FP32 inputs, so the same tree and decisions);
* the cloud-in-cell surface density and its adjoint against the FP64 oracle;
* the K-step gradient (64 KDK steps, checkpoints every 8) of a linear
  functional and of the surface-density loss, with respect to the initial
  positions, velocities and masses, against the oracle's reverse sweep and
  against central finite differences of the oracle's frozen-decision map;
* in the theta -> 0 limit, against the gradient of the FP64 direct sum.

The oracle follows its own FP64 trajectory; the trees along it are those of
the FP32-rounded positions, as on the GPU, which keeps the FP64 position
master for these runs.
"""
import numpy as np
import pytest

from gpu_util import device, rel_err, to_dev
from workloads import ics

pytestmark = pytest.mark.gpu


def _dev_tree(n, **kw):
    from paper_1412_0659_amd import Tree
    device()
    return Tree(n, adjoint=True, **kw)


def _zeros(*shape):
    import torch
    return torch.zeros(*shape, dtype=torch.float32, device="cuda")


@pytest.mark.parametrize("case", [("disk_halo", 0.4, 0.005), ("plummer", 0.7, 0.01),
                                  ("disk_halo", 1e-6, 0.01)])
def test_force_vjp_matches_oracle(oracle, case):
    model, theta, eps = case
    n = 2048 if theta < 1e-3 else 20000
    s = ics.disk_halo_scaled(n, 51) if model == "disk_halo" else ics.plummer(n, 52)
    rng = np.random.default_rng(53)
    u = rng.normal(size=(n, 3)).astype(np.float32)
    t = _dev_tree(n)
    t.build(to_dev(s.pos), to_dev(s.mass))
    gp, gm = _zeros(n, 3), _zeros(n)
    t.force_vjp(theta, eps, to_dev(u), 1.0, gp, gm)
    t.sync()
    gp1, gm1 = gp.cpu().numpy().astype(np.float64), gm.cpu().numpy().astype(np.float64)
    # coef scales and the outputs accumulate
    t.force_vjp(theta, eps, to_dev(u), 0.5, gp, gm)
    t.sync()
    assert np.allclose(gp.cpu().numpy(), 1.5 * gp1, rtol=1e-5, atol=1e-6 * np.abs(gp1).max())
    t.close()

    d = oracle.record_decisions(oracle.build_tree(s.pos, s.mass), theta)
    gx_ref, gm_ref = oracle.frozen_force_vjp(d, s.pos, s.mass, eps, u)
    ex = rel_err(gp1, gx_ref)
    em = rel_err(gm1, gm_ref)
    print(f"force vjp {case}: pos med {np.median(ex):.2e} p99 {np.percentile(ex, 99):.2e}; "
          f"mass med {np.median(em):.2e} p99 {np.percentile(em, 99):.2e}")
    assert np.median(ex) <= 1e-5 and np.percentile(ex, 99) <= 1e-4
    assert np.median(em) <= 1e-5 and np.percentile(em, 99) <= 1e-4
    dd = rng.normal(size=(n, 3))
    assert abs((gp1 * dd).sum() - (gx_ref * dd).sum()) <= 1e-5 * np.abs(gx_ref * dd).sum()


GRID = (0.2, 4.0, 16, 32)


def _near_seam(pos, grid, tol=1e-4):
    """Particles whose CIC cell choice FP32 rounding may flip."""
    r0, r1, nr, nphi = grid
    R = np.hypot(pos[:, 0], pos[:, 1])
    phi = np.mod(np.arctan2(pos[:, 1], pos[:, 0]), 2 * np.pi)
    u = (R - r0) / ((r1 - r0) / nr) - 0.5
    v = phi / (2 * np.pi / nphi) - 0.5
    frac = lambda a: np.abs(a - np.round(a))
    return (frac(u) < tol) | (frac(v) < tol) | (np.abs(R - r0) < tol) | (np.abs(R - r1) < tol)


def test_surface_density_and_vjp_match_oracle(oracle):
    import torch
    from paper_1412_0659_amd import binding as B
    s = ics.disk_halo(6000, 6000, 54)
    n = s.n
    t = _dev_tree(n)
    sel = torch.from_numpy(s.is_disk.astype(np.uint8)).to(device())
    pos, mass = to_dev(s.pos), to_dev(s.mass)
    sig = torch.empty(GRID[2], GRID[3], dtype=torch.float32, device="cuda")
    B.bh_cic_density(t.ctx, pos, mass, sel, GRID, sig)
    ref = oracle.cic_density(s.pos, s.mass, s.is_disk, GRID)
    got = sig.cpu().numpy().astype(np.float64)
    assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()
    B.bh_cic_density(t.ctx, pos, mass, None, GRID, sig)
    ref_all = oracle.cic_density(s.pos, s.mass, None, GRID)
    assert np.abs(sig.cpu().numpy() - ref_all).max() <= 1e-5 * np.abs(ref_all).max()

    g = np.random.default_rng(55).normal(size=GRID[2:]).astype(np.float32)
    gp, gm = _zeros(n, 3), _zeros(n)
    B.bh_cic_density_vjp(t.ctx, pos, mass, sel, GRID, to_dev(g), gp, gm)
    t.sync()
    gx_ref, gm_ref = oracle.cic_density_vjp(s.pos, s.mass, s.is_disk, GRID, g)
    ok = ~_near_seam(s.pos.astype(np.float64), GRID)
    gp, gm = gp.cpu().numpy(), gm.cpu().numpy()
    assert not gp[~s.is_disk].any() and not gm[~s.is_disk].any()
    scale = np.abs(gx_ref).max()
    assert np.abs(gp[ok] - gx_ref[ok]).max() <= 1e-4 * scale
    assert np.abs(gm[ok] - gm_ref[ok]).max() <= 1e-4 * np.abs(gm_ref).max()
    t.close()


# --- K-step gradients -----------------------------------------------------------

W = ics.DIFF_WORKLOADS["disk_halo_4096_adjoint"]


def _gpu_grad(s, loss_fn, theta, steps, every):
    import torch
    from paper_1412_0659_amd.autograd import leapfrog
    n = s.n
    t = _dev_tree(n, pos_fp64=True)
    x0 = to_dev(s.pos).requires_grad_(True)
    v0 = to_dev(s.vel).requires_grad_(True)
    m = to_dev(s.mass).requires_grad_(True)
    xK, vK = leapfrog(x0, v0, m, t, W["dt"], steps, theta, W["eps"], every)
    L = loss_fn(xK, vK, m, t)
    L.backward()
    torch.cuda.synchronize()
    out = [a.grad.cpu().numpy().astype(np.float64) for a in (x0, v0, m)]
    t.close()
    return out


def _oracle_decisions(oracle, s, theta, steps):
    m = s.mass.astype(np.float64)
    if theta < 1e-3:
        force = oracle.direct_force_fn(m, W["eps"])
    else:
        force = oracle.tree_force_fn(s.mass, theta, W["eps"])
    poss = oracle.kdk_positions(s.pos, s.vel, s.mass, W["dt"], steps, force)
    return oracle.trajectory_decisions(poss, s.mass, theta)


def _directional(g, d):
    return sum((a * b).sum() for a, b in zip(g, d))


def _check_fd(oracle_loss, s, g_gpu, rng, ndir, tol):
    m = s.mass.astype(np.float64)
    x0, v0 = s.pos.astype(np.float64), s.vel.astype(np.float64)
    for _ in range(ndir):
        d = (rng.normal(size=x0.shape), rng.normal(size=v0.shape) * 0.3, rng.normal(size=m.shape) * m)
        h = 1e-6
        fd = (oracle_loss(x0 + h * d[0], v0 + h * d[1], m + h * d[2])
              - oracle_loss(x0 - h * d[0], v0 - h * d[1], m - h * d[2])) / (2 * h)
        an = _directional(g_gpu, d)
        print(f"  FD {fd:.9e}  GPU adjoint {an:.9e}  rel {abs(fd - an) / abs(fd):.2e}")
        assert abs(fd - an) <= tol * abs(fd)


def _vec_err(g_gpu, g_ref):
    num = np.sqrt(sum(((a - b) ** 2).sum() for a, b in zip(g_gpu, g_ref)))
    return num / np.sqrt(sum((b ** 2).sum() for b in g_ref))


def test_leapfrog_gradient_of_linear_functional(oracle):
    import torch
    s = ics.disk_halo_scaled(W["n"], W["seed"])
    theta, K, every = W["theta"], W["steps"], W["every"]
    rng = np.random.default_rng(56)
    wx, wv = rng.normal(size=(s.n, 3)), rng.normal(size=(s.n, 3))
    wx_d, wv_d = to_dev(wx), to_dev(wv)
    g_gpu = _gpu_grad(s, lambda xK, vK, m, t: (xK * wx_d).sum() + (vK * wv_d).sum(), theta, K,
                      every)
    decs = _oracle_decisions(oracle, s, theta, K)
    m = s.mass.astype(np.float64)
    g_ref = oracle.leapfrog_frozen_vjp(s.pos, s.vel, m, W["dt"], decs, W["eps"], wx, wv)
    err = _vec_err(g_gpu, g_ref)
    print(f"linear functional: gradient vector rel err {err:.2e}")
    assert err <= 1e-4

    def L(x0, v0, mm):
        xK, vK, _ = oracle.leapfrog_frozen(x0, v0, mm, W["dt"], decs, W["eps"])
        return (wx * xK).sum() + (wv * vK).sum()

    _check_fd(L, s, g_gpu, rng, 3, 1e-4)


def _loss_parts(oracle, s, theta):
    """Target density (oracle, from the perturbed initial conditions) and the
    oracle's loss / gradient on the frozen decisions of its own trajectory."""
    K, grid, eps, dt = W["steps"], W["grid"], W["eps"], W["dt"]
    tgt_ic = ics.perturbed(s, W["target_seed"])
    m = s.mass.astype(np.float64)
    xt, _ = oracle.leapfrog(tgt_ic.pos, tgt_ic.vel, m, dt, K,
                            oracle.tree_force_fn(s.mass, 0.4, eps))
    target = oracle.cic_density(xt, m, s.is_disk, grid)
    decs = _oracle_decisions(oracle, s, theta, K)

    def loss(x0, v0, mm):
        xK, _, _ = oracle.leapfrog_frozen(x0, v0, mm, dt, decs, eps)
        return ((oracle.cic_density(xK, mm, s.is_disk, grid) - target) ** 2).sum()

    def grad():
        x0, v0 = s.pos.astype(np.float64), s.vel.astype(np.float64)
        xK, _, _ = oracle.leapfrog_frozen(x0, v0, m, dt, decs, eps)
        gsig = 2 * (oracle.cic_density(xK, m, s.is_disk, grid) - target)
        gxK, gmK = oracle.cic_density_vjp(xK, m, s.is_disk, grid, gsig)
        gx, gv, gm = oracle.leapfrog_frozen_vjp(x0, v0, m, dt, decs, eps, gxK, np.zeros_like(gxK))
        return gx, gv, gm + gmK

    return target, loss, grad


def _gpu_loss_grad(s, target, theta):
    import torch
    from paper_1412_0659_amd.autograd import surface_density
    sel = torch.from_numpy(s.is_disk.astype(np.uint8)).to(device())
    tgt = to_dev(target)

    def fn(xK, vK, m, t):
        sig = surface_density(xK, m, sel, t, W["grid"])
        return ((sig - tgt) ** 2).sum()

    return _gpu_grad(s, fn, theta, W["steps"], W["every"])


def test_surface_density_loss_gradient(oracle):
    s = ics.disk_halo_scaled(W["n"], W["seed"])
    target, loss, grad = _loss_parts(oracle, s, W["theta"])
    g_gpu = _gpu_loss_grad(s, target, W["theta"])
    g_ref = grad()
    err = _vec_err(g_gpu, g_ref)
    print(f"surface-density loss: gradient vector rel err {err:.2e}")
    assert err <= 1e-3
    _check_fd(loss, s, g_gpu, np.random.default_rng(57), 3, 1e-4)


def test_surface_density_loss_gradient_direct_limit(oracle):
    """theta -> 0: every decision a p-p pair; the GPU gradient is that of the
    FP64 direct-sum leapfrog."""
    s = ics.disk_halo_scaled(W["n"], W["seed"])
    target, loss, grad = _loss_parts(oracle, s, 1e-6)
    g_gpu = _gpu_loss_grad(s, target, 1e-6)
    g_ref = grad()
    err = _vec_err(g_gpu, g_ref)
    print(f"surface-density loss, direct limit: gradient vector rel err {err:.2e}")
    assert err <= 1e-3
    _check_fd(loss, s, g_gpu, np.random.default_rng(58), 1, 1e-4)
