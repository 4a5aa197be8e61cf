"""Parity of the differentiation form on the GPU against the oracle.

* tree_force_vjp against the oracle's hand-written adjoint of the
  frozen-decision force (same FP32 inputs, so the same tree and decisions);
* the cloud-in-cell surface density and its adjoint against the FP64 oracle;
* the K-step gradient (64 KDK steps, checkpoints every 8) of a linear
  functional and of the surface-density loss, with respect to the initial
  positions, velocities and masses, each array element by element against
  the oracle's reverse sweep, and along 16 directions (one perturbing only
  the masses) against central finite differences of the oracle's
  frozen-decision map;
* in the theta -> 0 limit, against the gradient of the FP64 direct sum;
* per theta, the tree gradient against the FP64 direct-sum gradient;
* the C ABI's segment sweep against one assembled from per-step calls.

The oracle follows its own FP64 trajectory; the trees along it are those of
the FP32-rounded positions, as on the GPU, which keeps the FP64 position
master for these runs.
"""
import numpy as np
import pytest

from gpu_util import device, paired_groups, rel_err, to_dev
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


def test_force_vjp_paired_target_sets(oracle):
    """The force VJP on a context with paired target sets (pair_groups = 48)
    against the oracle's adjoint over the same merged sets."""
    n, theta, eps = 20000, 0.4, 0.005
    s = ics.disk_halo_scaled(n, 51)
    u = np.random.default_rng(53).normal(size=(n, 3)).astype(np.float32)
    t = _dev_tree(n, pair_groups=48)
    t.build(to_dev(s.pos), to_dev(s.mass))
    gp, gm = _zeros(n, 3), _zeros(n)
    t.force_vjp(theta, eps, to_dev(u), 1.0, gp, gm)
    t.sync()
    ng = t.stats()["ngroups"]
    gp, gm = gp.cpu().numpy().astype(np.float64), gm.cpu().numpy().astype(np.float64)
    t.close()
    ot = paired_groups(oracle, oracle.build_tree(s.pos, s.mass), 48)
    assert ng == ot.ngroups
    gx_ref, gm_ref = oracle.frozen_force_vjp(oracle.record_decisions(ot, theta), s.pos, s.mass,
                                             eps, u)
    ex, em = rel_err(gp, gx_ref), rel_err(gm, gm_ref)
    print(f"paired force vjp: pos med {np.median(ex):.2e} p99 {np.percentile(ex, 99):.2e}; "
          f"mass med {np.median(em):.2e} p99 {np.percentile(em, 99):.2e}")
    assert np.median(ex) <= 1e-5 and np.percentile(ex, 99) <= 1e-4
    assert np.median(em) <= 1e-5 and np.percentile(em, 99) <= 1e-4


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


NAMES = ("g_x0", "g_v0", "g_m")


def _directional(g, d):
    return sum((a * b).sum() for a, b in zip(g, d))


def _fd_directions(s, rng, ndir):
    """ndir directions (dx0, dv0, dm): the first perturbs only the masses,
    the second only the positions, the third only the velocities; the rest
    all three."""
    m = s.mass.astype(np.float64)
    out = []
    for k in range(ndir):
        dx = rng.normal(size=(s.n, 3))
        dv = rng.normal(size=(s.n, 3)) * 0.3
        dm = rng.normal(size=s.n) * m
        if k == 0:
            dx, dv = dx * 0, dv * 0
        elif k == 1:
            dv, dm = dv * 0, dm * 0
        elif k == 2:
            dx, dm = dx * 0, dm * 0
        out.append((dx, dv, dm))
    return out


def _check_fd(oracle_loss, s, g_gpu, g_ref, rng, ndir, tol):
    """Directional derivatives of the GPU gradient against central finite
    differences of the oracle's frozen-decision map (FP64).

    The error is relative to max(|fd|, rms), rms being the root mean square
    of g . d over random directions with d's per-array norms,
    sqrt(sum_b |g_b|^2 |d_b|^2 / D_b) (b over x0, v0, m; D_b components;
    g the oracle's reverse-sweep gradient).  For a typical direction this is
    |fd| itself; it keeps a direction that happens to be nearly orthogonal
    to the gradient (|fd| far below rms) from dividing the gradient's error
    by a near-zero derivative."""
    m = s.mass.astype(np.float64)
    x0, v0 = s.pos.astype(np.float64), s.vel.astype(np.float64)
    worst = 0.0
    for k, d in enumerate(_fd_directions(s, rng, ndir)):
        h = 1e-6
        fd = (oracle_loss(x0 + h * d[0], v0 + h * d[1], m + h * d[2])
              - oracle_loss(x0 - h * d[0], v0 - h * d[1], m - h * d[2])) / (2 * h)
        an = _directional(g_gpu, d)
        rms = np.sqrt(sum(np.sum(np.square(g)) * np.sum(np.square(db)) / db.size
                          for g, db in zip(g_ref, d)))
        rel = abs(fd - an) / max(abs(fd), rms)
        worst = max(worst, rel)
        print(f"  FD dir {k:2d}: {fd:.9e}  GPU adjoint {an:.9e}  rms {rms:.3e}  rel {rel:.2e}")
        assert rel <= tol, (k, fd, an, rms)
    print(f"  FD: {ndir} directions, worst rel {worst:.2e}")


def _per_array(g_gpu, g_ref, floor_frac=1e-3):
    """For each of g_x0, g_v0, g_m: relative L2 error of the whole array and
    the per-particle relative error |g_i - ref_i| / max(|ref_i|, floor), the
    floor being floor_frac of the array's largest per-particle norm."""
    out = {}
    for name, a, b in zip(NAMES, g_gpu, g_ref):
        a2 = np.asarray(a, np.float64).reshape(len(a), -1)
        b2 = np.asarray(b, np.float64).reshape(len(b), -1)
        l2 = np.linalg.norm(a2 - b2) / np.linalg.norm(b2)
        nb = np.linalg.norm(b2, axis=1)
        e = np.linalg.norm(a2 - b2, axis=1) / np.maximum(nb, floor_frac * nb.max())
        out[name] = (l2, float(np.median(e)), float(np.percentile(e, 99)))
    return out


def _gate_per_array(label, g_gpu, g_ref, l2_tol=1e-4, med_tol=1e-4, p99_tol=1e-3):
    """Each array separately: relative L2 <= 1e-4, per-particle median <=
    1e-4 and 99th percentile <= 1e-3 (the force bar's 1:10 median:p99
    ratio)."""
    errs = _per_array(g_gpu, g_ref)
    for name, (l2, med, p99) in errs.items():
        print(f"{label} {name}: rel L2 {l2:.2e}, per-particle median {med:.2e} p99 {p99:.2e}")
    for name, (l2, med, p99) in errs.items():
        assert l2 <= l2_tol and med <= med_tol and p99 <= p99_tol, (label, name, l2, med, p99)
    return errs


def test_leapfrog_gradient_of_linear_functional(oracle):
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
    _gate_per_array("linear functional", g_gpu, g_ref)

    def L(x0, v0, mm):
        xK, vK, _ = oracle.leapfrog_frozen(x0, v0, mm, W["dt"], decs, W["eps"])
        return (wx * xK).sum() + (wv * vK).sum()

    _check_fd(L, s, g_gpu, g_ref, rng, 16, 1e-4)


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


def _gpu_loss_grad(s, target, theta, every=None):
    import torch
    from paper_1412_0659_amd.autograd import surface_density
    sel = torch.from_numpy(s.is_disk.astype(np.uint8)).to(device())
    tgt = to_dev(target)

    def fn(xK, vK, m, t):
        sig = surface_density(xK, m, sel, t, W["grid"])
        return ((sig - tgt) ** 2).sum()

    return _gpu_grad(s, fn, theta, W["steps"], W["every"] if every is None else every)


def test_surface_density_loss_gradient(oracle):
    s = ics.disk_halo_scaled(W["n"], W["seed"])
    target, loss, grad = _loss_parts(oracle, s, W["theta"])
    g_gpu = _gpu_loss_grad(s, target, W["theta"])
    g_ref = grad()
    _gate_per_array("surface-density loss", g_gpu, g_ref)
    _check_fd(loss, s, g_gpu, g_ref, np.random.default_rng(57), 16, 1e-4)


def test_surface_density_loss_gradient_direct_limit(oracle):
    """theta -> 0: every decision a p-p pair; the GPU gradient is that of the
    FP64 direct-sum leapfrog, gated at 1e-4 per array."""
    s = ics.disk_halo_scaled(W["n"], W["seed"])
    target, loss, grad = _loss_parts(oracle, s, 1e-6)
    g_gpu = _gpu_loss_grad(s, target, 1e-6)
    g_ref = grad()
    _gate_per_array("surface-density loss, direct limit", g_gpu, g_ref)
    _check_fd(loss, s, g_gpu, g_ref, np.random.default_rng(58), 16, 1e-4)


def _cos_l2(a, b):
    a, b = np.asarray(a).reshape(-1), np.asarray(b).reshape(-1)
    return (float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b))),
            float(np.linalg.norm(a - b) / np.linalg.norm(b)))


def test_tree_gradient_against_direct_sum_per_theta(oracle):
    """Per theta in {0.3, 0.4, 0.6}: the tree-code's 64-step gradient against
    the FP64 direct-sum gradient (cosine and relative L2 per array), for the
    surface-density loss and for w . v_K.  The latter's gradient with respect
    to x_0 and m comes only through the forces, so it shows the opening-angle
    error, where the density loss's gradient is dominated by the drift.
    Reported for the GPU and for the oracle's FP64 tree; gated: the GPU
    gradient within 1e-4 (relative L2 per array) of the oracle's at the same
    theta, and the oracle tree's distance from the direct-sum gradient growing
    with theta."""
    s = ics.disk_halo_scaled(W["n"], W["seed"])
    m = s.mass.astype(np.float64)
    dt, K, eps = W["dt"], W["steps"], W["eps"]
    w = np.random.default_rng(60).normal(size=(s.n, 3))
    w_d = to_dev(w)
    zero = np.zeros_like(w)

    def oracle_grad(theta):
        decs = _oracle_decisions(oracle, s, theta, K)
        return oracle.leapfrog_frozen_vjp(s.pos, s.vel, m, dt, decs, eps, zero, w)

    g_dir = oracle_grad(1e-6)
    target, _, sd_grad = _loss_parts(oracle, s, 1e-6)
    sd_dir = sd_grad()
    prev = None
    for theta in (0.3, 0.4, 0.6):
        g_gpu = _gpu_grad(s, lambda xK, vK, mm, t: (vK * w_d).sum(), theta, K, W["every"])
        g_orc = oracle_grad(theta)
        sd_gpu = _gpu_loss_grad(s, target, theta)
        errs = []
        for name, a, b, c, d in zip(NAMES, g_gpu, g_orc, g_dir, sd_gpu):
            cg, lg = _cos_l2(a, c)
            co, lo = _cos_l2(b, c)
            _, lgo = _cos_l2(a, b)
            cs, ls = _cos_l2(d, sd_dir[NAMES.index(name)])
            print(f"theta {theta} {name}: w.v_K vs direct-sum gradient: GPU cosine {cg:.8f} rel L2 "
                  f"{lg:.2e}; oracle tree cosine {co:.8f} rel L2 {lo:.2e}; GPU vs oracle tree "
                  f"{lgo:.2e} | density loss, GPU vs direct: cosine {cs:.8f} rel L2 {ls:.2e}")
            assert lgo <= 1e-4, (theta, name, lgo)
            errs.append(lo)
        if prev is not None:
            assert errs[0] > prev[0] and errs[2] > prev[2], (theta, errs, prev)
        prev = errs


def test_vjp_segment_matches_per_step_sweep():
    """leapfrog_vjp_segment drives the 64-step gradient through the C ABI
    alone (checkpoints every 8); it matches a sweep assembled from the
    per-step entry points (bh_load_state, tree_force_vjp,
    leapfrog_vjp_drift) over a snapshot of every step, and the autograd
    path, to the FP64 atomics' rounding."""
    import torch
    from paper_1412_0659_amd import binding as B
    from paper_1412_0659_amd.autograd import leapfrog
    s = ics.disk_halo_scaled(W["n"], W["seed"])
    n, K, every, dt, theta, eps = s.n, W["steps"], W["every"], W["dt"], W["theta"], W["eps"]
    rng = np.random.default_rng(59)
    wx, wv = rng.normal(size=(n, 3)).astype(np.float32), rng.normal(size=(n, 3)).astype(np.float32)
    t = _dev_tree(n, pos_fp64=True)
    ctx = t.ctx
    B.bh_set_state(ctx, to_dev(s.pos), to_dev(s.vel), to_dev(s.mass))
    nb = B.bh_state_bytes(ctx)

    def snap():
        buf = torch.empty(nb, dtype=torch.uint8, device="cuda")
        B.bh_save_state(ctx, buf)
        return buf

    snaps = [snap()]
    for _ in range(K):
        B.leapfrog_step(ctx, dt, theta, eps)
        snaps.append(snap())
    # (a) segments of 8 through the C ABI
    gx, gv, gm = to_dev(wx).clone(), to_dev(wv).clone(), _zeros(n)
    for s0 in reversed(range(0, K, every)):
        s1 = min(s0 + every, K)
        flags = (B.BH_SEG_FIRST if s0 == 0 else 0) | (B.BH_SEG_LAST if s1 == K else 0)
        B.leapfrog_vjp_segment(ctx, snaps[s0], n, s1 - s0, flags, dt, theta, eps, gx, gv, gm=gm)
    # separate output buffers leave the inputs untouched
    gx1, gv1, gx2, gv2 = to_dev(wx).clone(), to_dev(wv).clone(), _zeros(n, 3), _zeros(n, 3)
    B.leapfrog_vjp_segment(ctx, snaps[K - 1], n, 1, B.BH_SEG_LAST, dt, theta, eps, gx1, gv1, gx2,
                           gv2, None)
    t.sync()
    assert np.array_equal(gx1.cpu().numpy(), wx) and np.array_equal(gv1.cpu().numpy(), wv)
    # (b) the same sweep from the per-step entry points
    rx, rv, rm = to_dev(wx).clone(), to_dev(wv).clone(), _zeros(n)
    B.bh_load_state(ctx, snaps[K], n)
    B.tree_force_vjp(ctx, theta, eps, rv, 0.5 * dt, rx, rm)
    for j in reversed(range(K)):
        B.leapfrog_vjp_drift(ctx, dt, rx, rv)
        B.bh_load_state(ctx, snaps[j], n)
        B.tree_force_vjp(ctx, theta, eps, rv, dt if j > 0 else 0.5 * dt, rx, rm)
    t.sync()
    seg = [a.cpu().numpy().astype(np.float64) for a in (gx, gv, gm)]
    ref = [a.cpu().numpy().astype(np.float64) for a in (rx, rv, rm)]
    for name, a, b in zip(NAMES, seg, ref):
        e = np.linalg.norm(a - b) / np.linalg.norm(b)
        print(f"segment vs per-step sweep {name}: rel L2 {e:.2e}")
        assert e <= 1e-6, (name, e)
    t.close()
    # (c) the autograd path (which calls leapfrog_vjp_segment per checkpoint)
    wx_d, wv_d = to_dev(wx), to_dev(wv)
    g_auto = _gpu_grad(s, lambda xK, vK, m, tt: (xK * wx_d).sum() + (vK * wv_d).sum(), theta, K,
                       every)
    for name, a, b in zip(NAMES, g_auto, ref):
        e = np.linalg.norm(a - b) / np.linalg.norm(b)
        print(f"autograd vs per-step sweep {name}: rel L2 {e:.2e}")
        assert e <= 1e-6, (name, e)
    # argument checks (the tree is held in a name: a temporary would be
    # destroyed, and its context freed, before the call)
    t2 = _dev_tree(n, pos_fp64=True)
    with pytest.raises(B.BhError):
        B.leapfrog_vjp_segment(t2.ctx, snaps[0], n, 0, 0, dt, theta, eps, gx, gv)
    t2.close()
