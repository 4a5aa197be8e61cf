"""Pins of the oracle's multi-domain steps (Sec. III.B): the flop-weighted
cut of the curve, trees keyed in a given box, boundary trees, the cells of
a remote tree that a domain's targets reach (local essential tree) and the
walk of a remote tree.  Each is pinned by something other than itself: a
worked example of the cut, the defining inequalities of the cut, the exact
key relation of a doubled box, the direct sum the remote walk reduces to at
vanishing opening angle, and bit-identical FP64 forces when a remote tree
is cut down to the reached cells (with a planted omission that must show)."""
import numpy as np
import pytest

from oracle import let as LT
from workloads import ics


def _disk(n, seed=3):
    s = ics.disk_halo_scaled(n, seed=seed)
    return s.pos.astype(np.float32), s.mass.astype(np.float32)


def _clusters(n_per, seed=7):
    """Four uniform unit balls 40 apart, equal masses: remote domains that a
    boundary tree describes well enough."""
    rng = np.random.default_rng(seed)
    parts = []
    for c in ([0, 0, 0], [40, 0, 0], [0, 40, 0], [0, 0, 40]):
        v = rng.normal(size=(n_per, 3))
        r = rng.random(n_per) ** (1.0 / 3.0)
        parts.append(v / np.linalg.norm(v, axis=1, keepdims=True) * r[:, None] + c)
    pos = np.concatenate(parts).astype(np.float32)
    return pos, np.full(pos.shape[0], 1.0 / pos.shape[0], np.float32)


# --- the cut ----------------------------------------------------------------------

def test_decompose_worked_example():
    """n = 100, p = 4, cap 1.3 (C = 32); unit cost on the first 10 particles.
    Cost targets 2.5, 5, 7.5 give cuts 3, 5, 8; the cap moves them to
    4 (100 - 3 C = 4), 36 and 68."""
    cost = np.zeros(100, np.int64)
    cost[:10] = 1
    assert LT.decompose(cost, 4, 1.3).tolist() == [0, 4, 36, 68, 100]
    # without a binding cap: the cost targets themselves
    assert LT.decompose(cost, 4, 4.0).tolist() == [0, 3, 5, 8, 100]


@pytest.mark.parametrize("p", [1, 2, 3, 7, 16])
def test_decompose_defining_inequalities(p):
    rng = np.random.default_rng(100 + p)
    cost = rng.integers(1, 1000, size=3000).astype(np.int64)
    cuts = LT.decompose(cost, p, 100.0)        # cap never binds
    S = np.concatenate([[0], np.cumsum(cost)])
    W = int(S[-1])
    assert cuts[0] == 0 and cuts[-1] == cost.shape[0] and np.all(np.diff(cuts) >= 0)
    for j in range(1, p):
        i = int(cuts[j])
        assert int(S[i]) * p >= W * j            # the j/p share is reached at i
        assert i == 0 or int(S[i - 1]) * p < W * j   # and not one slot earlier
    share = np.add.reduceat(cost, cuts[:-1]) if p > 1 else np.array([W])
    assert np.all(np.abs(share - W / p) <= cost.max())


def test_decompose_cap():
    rng = np.random.default_rng(5)
    cost = np.ones(1000, np.int64)
    cost[:50] = rng.integers(1000, 5000, size=50)   # a costly clump at the start
    for p, cap in ((4, 1.3), (8, 1.1), (4, 1.0)):
        cuts = LT.decompose(cost, p, cap)
        C = int(np.floor(float(np.float32(cap)) * 1000 / p))
        assert np.all(np.diff(cuts) <= C) and cuts[-1] == 1000
    assert LT.decompose(np.ones(12, np.int64), 3, 1.0).tolist() == [0, 4, 8, 12]
    with pytest.raises(ValueError):
        LT.decompose(np.ones(10, np.int64), 3, 0.5)


def test_sampled_cut_worked_examples():
    """Keys 0..7, unit costs, two processes holding the even and the odd
    keys, two samples each: process 0 samples keys 0 and 4 (running cost
    1 >= 4/4 and 3 >= 12/4), process 1 keys 1 and 5; each sample weighs 4,
    so half the weight (8) lies before key 4: one boundary, key 4."""
    keys = np.arange(8, dtype=np.uint64)
    cuts, b = LT.decompose_sampled(keys, np.ones(8, np.int64), np.arange(8) % 2, 2, 1, 2, 2,
                                   1.3)
    assert cuts.tolist() == [0, 4, 8] and b.tolist() == [4]
    # keys 0..15 held by four processes (i mod 4), px = py = 2, two samples
    # per process and level: level-1 samples 0,1,2,3,8,9,10,11 (weight 4)
    # cut at key 8; the two pieces are cut at keys 2 and 10: slots 2, 8, 10.
    # The cap (C = floor(1.3 * 16 / 4) = 5) moves them to 2, 7, 11.
    keys = np.arange(16, dtype=np.uint64)
    cuts, b = LT.decompose_sampled(keys, np.ones(16, np.int64), np.arange(16) % 4, 2, 2, 2, 2,
                                   1.3)
    assert b.tolist() == [2, 8, 10] and cuts.tolist() == [0, 2, 7, 11, 16]
    cuts, _ = LT.decompose_sampled(keys, np.ones(16, np.int64), np.arange(16) % 4, 2, 2, 2, 2,
                                   4.0)
    assert cuts.tolist() == [0, 2, 8, 10, 16]


@pytest.mark.parametrize("px,py", [(1, 4), (2, 4), (4, 4), (3, 1)])
def test_sampled_cut_balances_cost(px, py):
    rng = np.random.default_rng(11 + px * py)
    n = 6000
    keys = np.sort(rng.integers(0, 2 ** 50, size=n).astype(np.uint64))
    keys[100:140] = keys[100]                  # a run of equal keys
    cost = rng.integers(1, 200, size=n).astype(np.int64)
    owner = rng.integers(0, px * py, size=n)
    p = px * py
    cuts, b = LT.decompose_sampled(keys, cost, owner, px, py, 256, 256, 4.0)
    assert np.all(np.diff(b.astype(np.float64)) >= 0) and np.all(np.diff(cuts) >= 0)
    share = np.add.reduceat(cost, cuts[:-1]) if p > 1 else np.array([cost.sum()])
    assert np.all(np.abs(share / (cost.sum() / p) - 1) < 0.06)
    for c in cuts[1:-1]:                         # equal keys stay together
        assert c == 0 or c == n or keys[c - 1] != keys[c]
    exact = LT.decompose(cost, p, 4.0)
    assert np.all(np.abs(cuts - exact) <= 0.03 * n / p)


# --- trees in a given box -----------------------------------------------------------

def test_box_equal_to_own_bbox(oracle):
    pos, mass = _disk(3000)
    t0 = oracle.build_tree(pos, mass)
    t1 = oracle.build_tree(pos, mass, box=(t0.lo, t0.side))
    assert np.array_equal(t0.skeys, t1.skeys) and np.array_equal(t0.perm, t1.perm)
    assert t0.cells["ncell"] == t1.cells["ncell"]
    assert np.array_equal(t0.mom["M"], t1.mom["M"])


def test_doubled_box_shifts_keys_one_digit(oracle):
    """Side 2s at the same corner: scale halves exactly, so every coordinate
    quantises to q >> 1 and every key loses its last digit (except where the
    own box clamped a coordinate at the far face to 2^21 - 1)."""
    pos, mass = _disk(3000)
    t0 = oracle.build_tree(pos, mass)
    lo, s, scale = oracle.fixed_box(t0.lo, 2 * t0.side)
    assert scale == t0.scale / 2
    k = oracle.morton_keys(pos, lo, scale)
    u = (pos - t0.lo) * t0.scale
    clamped = np.any(u >= np.float32(2 ** 21), axis=1)
    assert 1 <= clamped.sum() <= 3
    assert np.array_equal(k[~clamped], t0.keys[~clamped] >> np.uint64(3))


def test_box_clamps_outside_particles(oracle):
    pos = np.array([[-1, 0.5, 0.5], [2, 0.5, 0.5], [0.5, 0.5, 0.5]], np.float32)
    lo, side, scale = oracle.fixed_box([0, 0, 0], 1.0)
    k = oracle.morton_keys(pos, lo, scale)
    q = (1 << 21) - 1
    half = 1 << 20
    # x of particle 0 clamps to cell 0, of particle 1 to the last cell
    xs = [0, q, half]
    for key, x in zip(k, xs):
        got = 0
        for b in range(21):
            got |= int((int(key) >> (3 * b + 2)) & 1) << b
        assert got == x


# --- boundary trees -------------------------------------------------------------

@pytest.mark.parametrize("max_cells", [1, 16, 200, 10**6])
def test_boundary_partitions_particles(oracle, max_cells):
    pos, mass = _disk(8000)
    t = oracle.build_tree(pos, mass)
    L, inb, term = LT.boundary(t, max_cells)
    c = t.cells
    assert inb[0] and inb.sum() <= max(max_cells, 1)
    # every boundary cell's parent is a boundary cell, not terminal
    idx = np.nonzero(inb)[0][1:]
    assert np.all(inb[c["parent"][idx]]) and not np.any(term[c["parent"][idx]])
    # terminal cells: disjoint particle ranges covering all particles
    b = c["begin"][term]
    e = b + c["count"][term]
    order = np.argsort(b)
    assert b[order][0] == 0 and e[order][-1] == t.n
    assert np.array_equal(b[order][1:], e[order][:-1])
    # L is the deepest level that fits
    if L < 21:
        inb_all = np.ones(c["ncell"], bool)
        inb_all[1:] = c["count"][c["parent"][1:]] > 64
        assert (inb_all & (c["level"] <= L + 1)).sum() > max_cells


def test_boundary_boxes_hold_their_groups(oracle):
    pos, mass = _disk(8000)
    t = oracle.build_tree(pos, mass)
    box = (t.lo, t.side)
    L, inb, term = LT.boundary(t, 100)
    ids, bc, bh = LT.boundary_boxes(t, term, box)
    c = t.cells
    m = LT.margin(box)
    assert m > 0
    owner = np.zeros(t.n, np.int64)
    for k, i in enumerate(ids):
        owner[c["begin"][i]:c["begin"][i] + c["count"][i]] = k
    for g in range(t.ngroups):
        ks = owner[t.gbeg[g]:t.gbeg[g] + t.gcnt[g]]
        assert np.all(ks == ks[0])                  # inside one terminal cell
        k = ks[0]
        lo_g = t.gc[g] - t.gh[g]
        hi_g = t.gc[g] + t.gh[g]
        assert np.all(bc[k] - bh[k] <= lo_g - m / 2) and np.all(bc[k] + bh[k] >= hi_g + m / 2)


# --- remote walk and local essential trees ----------------------------------------

def test_remote_walk_small_theta_is_direct(oracle):
    """theta -> 0 opens every cell: the remote walk is the direct sum over the
    source particles (no self pair, all potential terms kept)."""
    pos, mass = _disk(1200)
    a, b = np.arange(0, 500), np.arange(500, 1200)
    box = (pos.min(0), float((pos.max(0) - pos.min(0)).max()))
    ta = oracle.build_tree(pos[a], mass[a], box=box)
    tb = oracle.build_tree(pos[b], mass[b], box=box)
    eps = 0.01
    acc, pot, npp, npc, _ = LT.walk_remote(ta, tb, 1e-6, eps)
    assert np.all(npc == 0) and np.all(npp == b.shape[0])
    x = pos[a].astype(np.float64)
    y = pos[b].astype(np.float64)
    d = y[None, :, :] - x[:, None, :]
    r2 = (d ** 2).sum(-1) + eps * eps
    ra = mass[b].astype(np.float64)[None, :] / r2 ** 1.5
    ref_acc = (d * ra[:, :, None]).sum(1)
    ref_pot = -(mass[b].astype(np.float64)[None, :] / np.sqrt(r2)).sum(1)
    assert np.max(np.abs(acc - ref_acc) / np.abs(ref_acc).max()) < 1e-12
    assert np.max(np.abs(pot - ref_pot) / np.abs(ref_pot)) < 1e-12


def _domains(pos, mass, p, curve="morton", theta=0.4, eps=0.01):
    from oracle import oracle as O
    g = O.build_tree(pos, mass, curve=curve)
    _, _, npp, npc = O.walk(g, theta, eps)
    cost = LT.particle_cost(g.n, g.gbeg, g.gcnt, npp, npc)
    cuts = LT.decompose(cost, p, 1.3)
    box = (g.lo, g.side)
    doms = [g.perm[cuts[d]:cuts[d + 1]] for d in range(p)]
    trees = [O.build_tree(pos[ix], mass[ix], box=box, curve=curve) for ix in doms]
    return g, cuts, box, doms, trees


@pytest.mark.parametrize("curve", ["morton", "ph"])
def test_let_walk_equals_full_remote_walk(oracle, curve):
    pos, mass = _disk(12000)
    theta, eps = 0.5, 0.01
    g, cuts, box, doms, trees = _domains(pos, mass, 4, curve, theta, eps)
    bnd = [LT.boundary(t, 128) for t in trees]
    for a in range(4):
        _, bc, bh = LT.boundary_boxes(trees[a], bnd[a][2], box)
        for b in range(4):
            if a == b:
                continue
            vis, opn, ins = LT.let_mark(trees[b], theta, bc, bh, bnd[b][2])
            assert ins == bool(np.any(opn & bnd[b][2]))
            assert np.all(vis[trees[b].cells["parent"][np.nonzero(vis)[0][1:]]])
            full = LT.walk_remote(trees[a], trees[b], theta, eps)
            cut = LT.walk_remote(trees[a], trees[b], theta, eps,
                                 cells=LT.prune(trees[b], vis, opn))
            for u, v in zip(full[:4], cut[:4]):
                assert np.array_equal(u, v)
            # a planted omission: one opened leaf loses its particles
            leaves = np.nonzero(opn & (trees[b].cells["nchild"] == 0))[0]
            if leaves.shape[0]:
                opn2 = opn.copy()
                opn2[leaves[0]] = False
                bad = LT.walk_remote(trees[a], trees[b], theta, eps,
                                     cells=LT.prune(trees[b], vis, opn2))
                assert not np.array_equal(full[0], bad[0])


def test_boundary_tree_suffices_for_far_domains(oracle):
    pos, mass = _clusters(3000)
    theta, eps = 0.5, 0.01
    g = oracle.build_tree(pos, mass)
    box = (g.lo, g.side)
    trees = [oracle.build_tree(pos[k * 3000:(k + 1) * 3000], mass[k * 3000:(k + 1) * 3000],
                               box=box) for k in range(4)]
    bnd = [LT.boundary(t, 64) for t in trees]
    suff = 0
    for a in range(4):
        _, bc, bh = LT.boundary_boxes(trees[a], bnd[a][2], box)
        for b in range(4):
            if a == b:
                continue
            vis, opn, ins = LT.let_mark(trees[b], theta, bc, bh, bnd[b][2])
            if ins:
                continue
            suff += 1
            L, inb, term = bnd[b]
            full = LT.walk_remote(trees[a], trees[b], theta, eps)
            cut = LT.walk_remote(trees[a], trees[b], theta, eps,
                                 cells=LT.prune(trees[b], inb, inb & ~term))
            for u, v in zip(full[:4], cut[:4]):
                assert np.array_equal(u, v)
    assert suff == 12


def test_domain_forces_match_one_tree(oracle):
    pos, mass = _disk(10000)
    theta, eps = 0.4, 0.01
    g, cuts, box, doms, trees = _domains(pos, mass, 4, "morton", theta, eps)
    acc, pot, _ = LT.domain_forces(pos, mass, doms, box, theta, eps)
    acc1, pot1, _, _ = oracle.walk(g, theta, eps)
    dacc, dpot = oracle.direct(pos, mass, eps)
    e1 = np.linalg.norm(acc - acc1, axis=1) / np.linalg.norm(dacc, axis=1)
    ed = np.linalg.norm(acc - dacc, axis=1) / np.linalg.norm(dacc, axis=1)
    e0 = np.linalg.norm(acc1 - dacc, axis=1) / np.linalg.norm(dacc, axis=1)
    # both tree forms carry the opening-angle error; neither is far off
    assert np.median(ed) < 2 * np.median(e0) + 1e-6 and np.percentile(ed, 99) < 1e-2
    assert np.median(e1) < 1e-3
    assert np.max(np.abs(pot - dpot) / np.abs(dpot)) < 1e-2
