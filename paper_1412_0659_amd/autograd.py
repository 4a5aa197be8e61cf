"""torch.autograd wrappers of the differentiation form.

``leapfrog`` runs K kick-drift-kick steps of the tree-code (Sec. III.B.2,
full rebuild per step) and differentiates the final state with respect to
the initial positions, velocities and masses, holding the walk's decisions
fixed.  Every arithmetic step runs in the HIP library: the forward steps
(leapfrog_step) and, per checkpoint segment, the reverse sweep
(leapfrog_vjp_segment: the segment's recomputation, the adjoints of the force
and of the drift).  Memory is bounded by checkpointing: an exact state
snapshot is kept every ``every`` steps and each segment is recomputed during
the backward sweep, reproducing bit-identical trees.

Reverse sweep of one step j (x_j -> x_{j+1}), with cotangents (gx, gv):
    gv += dt gx                         (drift)
    gx += c_j J(x_j)^T gv ; gm += c_j Jm(x_j)^T gv   (kicks at x_j)
with c_j = dt for 0 < j (the second kick of step j-1 and the first kick of
step j share the cotangent) and c_0 = dt/2; the second kick of the last step
contributes (dt/2) J(x_K)^T gv_K before the sweep.

``surface_density`` is the cloud-in-cell (R, phi) surface density of the
selected particles, the observable of the differentiation workload.
"""
from __future__ import annotations

import torch

from . import binding as B


class LeapfrogFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x0, v0, m, tree, dt, steps, theta, eps, every):
        tree.set_state(x0.detach().contiguous(), v0.detach().contiguous(),
                       m.detach().contiguous())
        ckpts = {0: tree.save()}
        for k in range(steps):
            tree.step(dt, theta, eps)
            if (k + 1) % every == 0 and k + 1 < steps:
                ckpts[k + 1] = tree.save()
        xK, vK = tree.state()
        ctx.tree, ctx.ckpts = tree, ckpts
        ctx.params = (float(dt), int(steps), float(theta), float(eps))
        return xK, vK

    @staticmethod
    def backward(ctx, gxK, gvK):
        tree = ctx.tree
        dt, steps, theta, eps = ctx.params
        n = tree.n
        dev = torch.device("cuda")
        gx = (gxK if gxK is not None else torch.zeros(n, 3, device=dev)).float().contiguous().clone()
        gv = (gvK if gvK is not None else torch.zeros(n, 3, device=dev)).float().contiguous().clone()
        gm = torch.zeros(n, device=dev, dtype=torch.float32)
        starts = sorted(ctx.ckpts)
        for si in reversed(range(len(starts)) if steps > 0 else ()):
            s0 = starts[si]
            s1 = starts[si + 1] if si + 1 < len(starts) else steps
            flags = (B.BH_SEG_FIRST if s0 == 0 else 0) | (B.BH_SEG_LAST if s1 == steps else 0)
            B.leapfrog_vjp_segment(tree.ctx, ctx.ckpts[s0], n, s1 - s0, flags, dt, theta, eps,
                                   gx, gv, gm=gm)
        return gx, gv, gm, None, None, None, None, None, None


def leapfrog(x0, v0, m, tree, dt, steps, theta, eps, every=8):
    """Differentiable K-step leapfrog: returns (x_K, v_K) in caller order."""
    return LeapfrogFn.apply(x0, v0, m, tree, dt, steps, theta, eps, every)


class SurfaceDensityFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, mass, sel, tree, grid):
        nr, nphi = grid[2], grid[3]
        out = torch.empty(nr, nphi, device=pos.device, dtype=torch.float32)
        p = pos.detach().contiguous()
        w = mass.detach().contiguous()
        B.bh_cic_density(tree.ctx, p, w, sel, grid, out)
        ctx.save_for_backward(p, w)
        ctx.sel, ctx.tree, ctx.grid = sel, tree, grid
        return out

    @staticmethod
    def backward(ctx, g):
        p, w = ctx.saved_tensors
        gp = torch.zeros_like(p)
        gw = torch.zeros_like(w)
        B.bh_cic_density_vjp(ctx.tree.ctx, p, w, ctx.sel, ctx.grid, g.float().contiguous(), gp,
                             gw)
        return gp, gw, None, None, None


def surface_density(pos, mass, sel, tree, grid):
    """Cloud-in-cell surface density on grid = (r_min, r_max, n_r, n_phi)."""
    return SurfaceDensityFn.apply(pos, mass, sel, tree, grid)
