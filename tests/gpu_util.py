"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
fetch its arrays; compare with the oracle."""
import numpy as np


def device():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch.device("cuda")


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device())


def gpu_tree(pos, mass, nleaf=16, ncrit=64, vel=None, far_fp16=False, curve="morton"):
    from paper_1412_0659_amd import Tree
    t = Tree(max(1, len(mass)), nleaf, ncrit, far_fp16, curve=curve)
    if vel is None:
        t.build(to_dev(pos), to_dev(mass))
    else:
        t.set_state(to_dev(pos), to_dev(vel), to_dev(mass))
    t.sync()
    return t


def gpu_force(t, theta, eps):
    acc, pot = t.force(theta, eps)
    t.sync()
    return acc.cpu().numpy().astype(np.float64), pot.cpu().numpy().astype(np.float64)


def cells_of(t):
    return {k: t.export("cell_" + k) for k in
            ("level", "prefix", "begin", "count", "child0", "nchild", "parent")}


def assert_tree_equal(t, ot):
    """Keys, permutation, cells and groups bit-exact against the oracle tree."""
    assert np.array_equal(t.export("keys"), ot.skeys)
    assert np.array_equal(t.export("perm").astype(np.int64), ot.perm)
    box = t.export("box")
    assert np.array_equal(box[:3], ot.lo) and box[3] == ot.side and box[4] == ot.scale
    c = cells_of(t)
    oc = ot.cells
    assert c["level"].shape[0] == oc["ncell"]
    assert np.array_equal(t.export("level_start").astype(np.int64), oc["level_start"])
    for k in ("level", "prefix", "begin", "count", "nchild"):
        assert np.array_equal(c[k].astype(np.int64), oc[k].astype(np.int64)), k
    internal = oc["nchild"] > 0
    assert np.array_equal(c["child0"][internal].astype(np.int64), oc["child0"][internal])
    par = c["parent"].astype(np.int64)
    par[0] = -1
    assert np.array_equal(par, oc["parent"])
    assert np.array_equal(t.export("group_begin").astype(np.int64), ot.gbeg)
    assert np.array_equal(t.export("group_count").astype(np.int64), ot.gcnt)


def rel_err(a, ref):
    a = np.asarray(a, np.float64)
    ref = np.asarray(ref, np.float64)
    if a.ndim == 1:
        return np.abs(a - ref) / np.abs(ref)
    return np.sqrt(((a - ref) ** 2).sum(1)) / np.sqrt((ref ** 2).sum(1))


def paired_groups(oracle, ot, cap):
    """The oracle tree with groups 2k and 2k + 1 merged when their cells are
    siblings and they hold at most cap particles together (boxes of the
    merged target sets recomputed)."""
    import dataclasses
    j = np.arange(1, ot.ngroups, 2)
    par = ot.cells["parent"][ot.gcell]
    keep = np.ones(ot.ngroups, bool)
    sib = (par[j - 1] == par[j]) & (ot.gcell[j - 1] != 0)
    keep[j[(ot.gcnt[j - 1] + ot.gcnt[j] <= cap) & sib]] = False
    gbeg = np.ascontiguousarray(ot.gbeg[keep])
    gcnt = np.diff(np.append(gbeg, ot.n)).astype(np.int64)
    gc, gh = oracle.group_boxes(gbeg, gcnt, ot.x, ot.y, ot.z)
    return dataclasses.replace(ot, gbeg=gbeg, gcnt=gcnt, gcell=ot.gcell[keep], gc=gc, gh=gh)
