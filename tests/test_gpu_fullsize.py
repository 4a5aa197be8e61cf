"""Parity at the benchmark's full sizes, in the launch configuration the
benchmark times (a context sized for the workload, the default walk grid).

The oracle builds the whole tree from the same seeded particles (integer
results and FP64 moments compared in full) and walks a seeded sample of
groups; the GPU's interaction counts and forces at those groups' targets
are compared one by one.  The precision form is checked at its 4M size
against the oracle's direct sum at sampled targets.
"""
import numpy as np
import pytest

from gpu_util import assert_tree_equal, gpu_force, gpu_tree, rel_err
from workloads import ics

pytestmark = pytest.mark.gpu

MED_TOL, P99_TOL = 1e-5, 1e-4


@pytest.mark.parametrize("name", ["disk_halo_13m", "disk_halo_1m"])
def test_full_size_tree_and_sampled_walk(oracle, name):
    w = ics.WORKLOADS[name]
    s = ics.make(name)
    print(f"case {name} n={s.n} theta={w['theta']} eps={w['eps']}", flush=True)
    t = gpu_tree(s.pos, s.mass)
    acc, pot = gpu_force(t, w["theta"], w["eps"])
    ot = oracle.build_tree(s.pos, s.mass)
    assert_tree_equal(t, ot)
    assert np.array_equal(t.export("mom_M"), ot.mom["M"])
    assert np.array_equal(t.export("mom_com"), ot.mom["com"])
    assert np.array_equal(t.export("mom_Q"), ot.mom["Q"])
    rng = np.random.default_rng(77)
    sel = np.sort(rng.choice(ot.ngroups, size=min(3000, ot.ngroups), replace=False))
    oacc, opot, onpp, onpc = oracle.walk(ot, w["theta"], w["eps"], groups=sel)
    assert np.array_equal(t.export("group_npp").astype(np.int64)[sel], onpp[sel])
    assert np.array_equal(t.export("group_npc").astype(np.int64)[sel], onpc[sel])
    tgt = np.concatenate([ot.perm[ot.gbeg[g]:ot.gbeg[g] + ot.gcnt[g]] for g in sel])
    ea = rel_err(acc[tgt], oacc[tgt])
    ep = rel_err(pot[tgt], opot[tgt])
    print(f"  {len(tgt)} targets: acc med {np.median(ea):.2e} p99 {np.percentile(ea, 99):.2e}  "
          f"pot med {np.median(ep):.2e} p99 {np.percentile(ep, 99):.2e}", flush=True)
    assert np.median(ea) <= MED_TOL and np.percentile(ea, 99) <= P99_TOL
    assert np.median(ep) <= MED_TOL and np.percentile(ep, 99) <= P99_TOL
    t.close()


def test_precision_form_full_size(oracle):
    """4M disk + halo, FP16 far field: at most 1e-3 median force error
    against the FP64 direct sum at 1000 sampled targets, for each theta."""
    w = ics.WORKLOADS["disk_halo_4m"]
    s = ics.make("disk_halo_4m")
    idx = ics.subsample(s.n, 1000, 40)
    eps32 = float(np.float32(w["eps"]))
    ra, rp = oracle.direct(s.pos, s.mass, eps32, idx)
    for theta in (0.3, 0.4, 0.6):
        row = []
        for f16 in (False, True):
            t = gpu_tree(s.pos, s.mass, far_fp16=f16)
            acc, pot = gpu_force(t, theta, w["eps"])
            t.close()
            ea = rel_err(acc[idx], ra)
            row.append((np.median(ea), np.percentile(ea, 99)))
        print(f"  theta {theta}: FP32 tree vs direct med {row[0][0]:.2e} p99 {row[0][1]:.2e}; "
              f"FP16 far med {row[1][0]:.2e} p99 {row[1][1]:.2e}", flush=True)
        assert row[1][0] <= 1e-3


def _group_subset(oracle, d, sel):
    """The decisions of the groups `sel` only (their lists, on the same tree
    topology): the frozen-decision VJP of a cotangent that is zero outside
    those groups' targets is the same computed over them alone."""
    import dataclasses
    t = d.tree
    npc = d.pc_off[sel + 1] - d.pc_off[sel]
    nlf = d.lf_off[sel + 1] - d.lf_off[sel]
    pc = np.concatenate([d.pc[d.pc_off[g]:d.pc_off[g + 1]] for g in sel])
    lf = np.concatenate([d.lf[d.lf_off[g]:d.lf_off[g + 1]] for g in sel])
    sub = dataclasses.replace(t, gbeg=np.ascontiguousarray(t.gbeg[sel]),
                              gcnt=np.ascontiguousarray(t.gcnt[sel]),
                              gcell=np.ascontiguousarray(t.gcell[sel]),
                              gc=np.ascontiguousarray(t.gc[sel]), gh=np.ascontiguousarray(t.gh[sel]))
    return oracle.Decisions(sub, np.concatenate([[0], np.cumsum(npc)]).astype(np.int64),
                            np.ascontiguousarray(pc, np.int64),
                            np.concatenate([[0], np.cumsum(nlf)]).astype(np.int64),
                            np.ascontiguousarray(lf, np.int64))


def test_force_vjp_full_size_sampled_targets(oracle):
    """The force VJP at the differentiation workload's full size (1M disk +
    halo, theta 0.4), in the launch configuration the benchmark times, for
    a cotangent that is nonzero only on the targets of 1500 seeded groups:
    every particle's gradient (targets, and sources through particle-particle
    terms and the cell moments) against the oracle's frozen-decision
    adjoint over those groups."""
    import torch
    from paper_1412_0659_amd import Tree
    w = ics.DIFF_WORKLOADS["disk_halo_1m_adjoint"]
    s = ics.disk_halo_scaled(w["n"], w["seed"])
    n = s.n
    print(f"case force vjp 1m n={n} theta={w['theta']} eps={w['eps']}", flush=True)
    ot = oracle.build_tree(s.pos, s.mass)
    d = oracle.record_decisions(ot, w["theta"])
    rng = np.random.default_rng(78)
    sel = np.sort(rng.choice(ot.ngroups, size=1500, replace=False))
    u = np.zeros((n, 3), np.float32)
    tgt = np.concatenate([ot.perm[ot.gbeg[g]:ot.gbeg[g] + ot.gcnt[g]] for g in sel])
    u[tgt] = rng.normal(size=(len(tgt), 3)).astype(np.float32)
    gx_ref, gm_ref = oracle.frozen_force_vjp(_group_subset(oracle, d, sel), s.pos, s.mass,
                                             w["eps"], u)
    t = Tree(n, adjoint=True)
    t.build(torch.from_numpy(s.pos).cuda(), torch.from_numpy(s.mass).cuda())
    gp = torch.zeros(n, 3, device="cuda")
    gm = torch.zeros(n, device="cuda")
    t.force_vjp(w["theta"], w["eps"], torch.from_numpy(u).cuda(), 1.0, gp, gm)
    t.sync()
    gp, gm = gp.cpu().numpy().astype(np.float64), gm.cpu().numpy().astype(np.float64)
    t.close()
    # every particle the sampled groups reach, with a floor at 1e-3 of the
    # largest gradient for the ones they barely reach
    for name, a, b in (("g_pos", gp, gx_ref), ("g_mass", gm, gm_ref)):
        a2, b2 = a.reshape(n, -1), b.reshape(n, -1)
        nb = np.linalg.norm(b2, axis=1)
        hit = nb > 0
        e = np.linalg.norm(a2 - b2, axis=1)[hit] / np.maximum(nb[hit], 1e-3 * nb.max())
        print(f"  {name}: {hit.sum()} particles reached, median {np.median(e):.2e} "
              f"p99 {np.percentile(e, 99):.2e}", flush=True)
        assert np.median(e) <= 1e-5 and np.percentile(e, 99) <= 1e-4, name
        assert not a2[~hit].any(), name
        # the sampled targets themselves, each against its own gradient's norm
        et = np.linalg.norm(a2[tgt] - b2[tgt], axis=1) / np.linalg.norm(b2[tgt], axis=1)
        print(f"  {name} at the {len(tgt)} sampled targets: median {np.median(et):.2e} "
              f"p99 {np.percentile(et, 99):.2e}", flush=True)
        assert np.median(et) <= 1e-5 and np.percentile(et, 99) <= 1e-4, name
