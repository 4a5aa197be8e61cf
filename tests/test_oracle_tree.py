"""Pins of the oracle's integer steps: keys, sort, octree build, groups, and
the moments of the upward pass (Sec. I.A, Sec. III.B.1, Sec. VI.A Eq. (1)).

Every check here compares the oracle with something other than itself:
hand-derived keys, a recursive geometric subdivision written from the
definition, or per-cell sums taken directly over the cell's particles.
"""
import numpy as np
import pytest

from golden_io import morton_sets
from workloads import ics


def test_morton_hand_examples(oracle):
    for name, pts in morton_sets().items():
        pos = np.array([p for p, _ in pts], np.float32)
        lo, side, scale = oracle.bbox(pos)
        keys = oracle.morton_keys(pos, lo, scale)
        want = np.array([k for _, k in pts], np.uint64)
        assert np.array_equal(keys, want), name


def test_bbox_definition(oracle):
    rng = np.random.default_rng(0)
    pos = (rng.normal(size=(1000, 3)) * [3.0, 1.0, 0.5] + [1, -2, 7]).astype(np.float32)
    lo, side, scale = oracle.bbox(pos)
    assert np.array_equal(lo, pos.min(0))
    ext = pos.max(0) - pos.min(0)
    assert side == ext.max()
    assert scale == np.float32(2.0 ** 21 / np.float64(side))
    # degenerate: all points coincide -> side 1
    lo1, side1, scale1 = oracle.bbox(np.ones((5, 3), np.float32))
    assert side1 == 1.0 and scale1 == np.float32(2.0 ** 21)


def _quantise(pos, lo, scale):
    t = (pos - lo).astype(np.float32)
    u = (t * np.float32(scale)).astype(np.float32)
    return np.minimum(u.astype(np.uint64), 2 ** 21 - 1)


def test_key_bits_are_interleaved_coordinates(oracle):
    """Bit 3b+2 / 3b+1 / 3b of the key is bit b of qx / qy / qz, with q the
    FP32 quantisation of the position (written here with numpy float32)."""
    s = ics.plummer(4096, 3)
    lo, side, scale = oracle.bbox(s.pos)
    keys = oracle.morton_keys(s.pos, lo, scale)
    q = _quantise(s.pos, lo, scale)
    for a in range(3):
        back = np.zeros_like(keys)
        for b in range(21):
            back |= ((keys >> np.uint64(3 * b + 2 - a)) & np.uint64(1)) << np.uint64(b)
        assert np.array_equal(back, q[:, a])


def test_sort_is_stable(oracle):
    keys = np.array([5, 3, 5, 1, 3, 3, 0, 5], np.uint64)
    perm = oracle.sort_keys(keys)
    assert list(perm) == [6, 3, 1, 4, 5, 0, 2, 7]


def _brute_octree(q, nleaf):
    """Recursive geometric subdivision on integer coordinates: a cube of
    side 2^(21 - l) at level l holding more than nleaf points (and l < 21) is
    cut into its 8 octants, octant digit = 4 bx + 2 by + bz.  Returns cells as
    (level, sorted tuple of point ids) in breadth-first, digit order."""
    out = []
    frontier = [(0, np.arange(q.shape[0]))]
    while frontier:
        nxt = []
        for lev, ids in frontier:
            out.append((lev, ids))
            if ids.size > nleaf and lev < 21:
                bit = 20 - lev
                b = (q[ids] >> np.uint64(bit)) & np.uint64(1)
                d = (b[:, 0] << np.uint64(2)) | (b[:, 1] << np.uint64(1)) | b[:, 2]
                for dig in range(8):
                    sub = ids[d == dig]
                    if sub.size:
                        nxt.append((lev + 1, sub))
        frontier = nxt
    return out


@pytest.mark.parametrize("case", ["plummer", "clustered", "duplicates"])
def test_build_equals_geometric_subdivision(oracle, case):
    rng = np.random.default_rng(11)
    if case == "plummer":
        pos = ics.plummer(1500, 5).pos
    elif case == "clustered":
        pos = np.concatenate([rng.normal(size=(600, 3)) * 1e-3, rng.uniform(-5, 5, (400, 3)),
                              rng.normal(size=(300, 3)) * 1e-5 + 2.0]).astype(np.float32)
    else:
        pos = np.concatenate([np.full((20, 3), 0.25), rng.uniform(0, 1, (100, 3))]).astype(np.float32)
    mass = np.ones(pos.shape[0], np.float32)
    t = oracle.build_tree(pos, mass)
    q = _quantise(pos, t.lo, t.scale)
    brute = _brute_octree(q, 16)
    c = t.cells
    assert c["ncell"] == len(brute)
    for i, (lev, ids) in enumerate(brute):
        assert c["level"][i] == lev
        got = np.sort(t.perm[c["begin"][i]:c["begin"][i] + c["count"][i]])
        assert np.array_equal(got, np.sort(ids))


def test_build_invariants_and_edge_cases(oracle):
    # N = 1: a single leaf root
    t = oracle.build_tree(np.zeros((1, 3), np.float32), np.ones(1, np.float32))
    assert t.cells["ncell"] == 1 and t.cells["nchild"][0] == 0 and t.ngroups == 1
    # 20 coincident points: one chain down to a level-21 leaf holding all 20
    t = oracle.build_tree(np.full((20, 3), 0.5, np.float32), np.ones(20, np.float32))
    c = t.cells
    assert c["ncell"] == 22 and c["level"][-1] == 21 and c["count"][-1] == 20
    # 100 coincident points: the level-21 leaf group is cut into chunks of 64
    t = oracle.build_tree(np.full((100, 3), 0.5, np.float32), np.ones(100, np.float32))
    assert list(t.gcnt) == [64, 36] and list(t.gbeg) == [0, 64]
    # general invariants
    s = ics.disk_halo(3000, 12000, 9)
    t = oracle.build_tree(s.pos, s.mass)
    c = t.cells
    leaf = c["nchild"] == 0
    assert np.all((c["count"][leaf] <= 16) | (c["level"][leaf] == 21))
    cover = np.zeros(t.n, np.int64)
    for b, n in zip(c["begin"][leaf], c["count"][leaf]):
        cover[b:b + n] += 1
    assert np.all(cover == 1)
    internal = np.nonzero(~leaf)[0]
    for p in internal:
        ch = slice(c["child0"][p], c["child0"][p] + c["nchild"][p])
        assert c["count"][ch].sum() == c["count"][p]
        assert np.all(c["parent"][ch] == p)
        assert np.all(c["prefix"][ch] >> np.uint64(3) == c["prefix"][p])
    assert np.all(np.diff(c["level"]) >= 0)
    # cell count within the stated capacity bound
    assert c["ncell"] <= oracle.cell_capacity(t.n)


def test_groups_definition(oracle):
    s = ics.disk_halo(3000, 12000, 9)
    t = oracle.build_tree(s.pos, s.mass)
    c = t.cells
    assert t.gbeg[0] == 0 and np.all(t.gbeg[1:] == t.gbeg[:-1] + t.gcnt[:-1])
    assert t.gcnt.sum() == t.n and t.gcnt.max() <= 64
    isgroup = np.zeros(c["ncell"], bool)
    for i in range(c["ncell"]):
        small = c["count"][i] <= 64 or c["nchild"][i] == 0
        top = i == 0 or c["count"][c["parent"][i]] > 64
        isgroup[i] = small and top
    assert set(np.nonzero(isgroup)[0]) == set(t.gcell)
    # boxes: tight FP32 boxes
    for g in range(0, t.ngroups, 37):
        sl = slice(t.gbeg[g], t.gbeg[g] + t.gcnt[g])
        for a, arr in enumerate((t.x, t.y, t.z)):
            mn, mx = arr[sl].min(), arr[sl].max()
            assert t.gc[g, a] == np.float32((mn + mx) * np.float32(0.5))
            assert t.gh[g, a] == np.float32((mx - mn) * np.float32(0.5))


def test_moments_bottom_up_equal_direct_sums(oracle):
    s = ics.disk_halo(3000, 12000, 9)
    t = oracle.build_tree(s.pos, s.mass)
    c, mo = t.cells, t.mom
    x = np.stack([t.x, t.y, t.z], 1).astype(np.float64)
    m = t.m.astype(np.float64)
    for i in list(range(0, c["ncell"], 53)) + [0]:
        sl = slice(c["begin"][i], c["begin"][i] + c["count"][i])
        M = m[sl].sum()
        com = (m[sl, None] * x[sl]).sum(0) / M
        d = x[sl] - com
        Q = np.einsum("i,ia,ib->ab", m[sl], d, d)
        q6 = np.array([Q[0, 0], Q[1, 1], Q[2, 2], Q[0, 1], Q[0, 2], Q[1, 2]])
        assert abs(mo["M"][i] - M) <= 1e-12 * M
        assert np.allclose(mo["com"][i], com, rtol=0, atol=1e-12 * (1 + np.abs(com).max()))
        assert np.allclose(mo["Q"][i], q6, rtol=1e-10, atol=1e-13 * M * (1 + (d ** 2).sum(1).max()))
    assert abs(mo["M"][0] - m.sum()) < 1e-12
    # geometry: level-l cell size and the offset of the centre of mass from the centre
    lev = c["level"]
    assert np.array_equal(mo["lf"], (t.side * np.float32(2.0) ** -lev.astype(np.float32)).astype(np.float32))
    # the centre of mass of a cell lies inside the cell: delta <= sqrt(3)/2 l
    assert np.all(mo["deltaf"] <= np.float32(0.8661) * mo["lf"] * (1 + 1e-5))


def test_paired_target_sets_helper(oracle):
    """The merged target sets the paired-group parity tests build from the
    oracle's groups: they partition the particles in key order, each holds
    at most the cap or is one original group, a merged set is exactly two
    consecutive sibling groups 2k, 2k + 1, and every such pair within the cap
    is merged."""
    import numpy as np
    from gpu_util import paired_groups
    from workloads import ics
    d = ics.disk_halo(4000, 16000, 12)
    ot = oracle.build_tree(d.pos, d.mass)
    par = ot.cells["parent"][ot.gcell]
    for cap in (2, 32, 48, 64):
        pt = paired_groups(oracle, ot, cap)
        assert pt.gbeg[0] == 0 and np.all(np.diff(pt.gbeg) > 0)
        assert np.array_equal(np.append(pt.gbeg[1:], ot.n) - pt.gbeg, pt.gcnt)
        starts = set(ot.gbeg.tolist())
        assert set(pt.gbeg.tolist()) <= starts
        dropped = sorted(starts - set(pt.gbeg.tolist()))
        idx = {b: k for k, b in enumerate(ot.gbeg.tolist())}
        for b in dropped:  # the start of group 2k + 1, merged into 2k
            j = idx[b]
            assert j % 2 == 1 and par[j] == par[j - 1] and ot.gcell[j - 1] != 0
            assert ot.gcnt[j - 1] + ot.gcnt[j] <= cap
        for j in range(1, ot.ngroups, 2):  # every qualifying pair is merged
            if par[j] == par[j - 1] and ot.gcell[j - 1] != 0 and ot.gcnt[j - 1] + ot.gcnt[j] <= cap:
                assert int(ot.gbeg[j]) in dropped
        gc, gh = oracle.group_boxes(pt.gbeg, pt.gcnt, ot.x, ot.y, ot.z)
        assert np.array_equal(gc, pt.gc) and np.array_equal(gh, pt.gh)
