"""Pins of the oracle's Peano-Hilbert keys (Sec. III.B.1 sorts particles
along a Peano-Hilbert curve) and the identity of the octree cell set under
the Peano-Hilbert and Morton orders.  The pins are properties that define a
Hilbert curve, independent of the encoding steps: the index is a bijection
of the grid, consecutive indices are face neighbours, every octant of every
level is one contiguous index range, and the curve starts at the origin."""
import numpy as np
import pytest

from workloads import ics


def _grid(bits):
    r = np.arange(1 << bits)
    return np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3).astype(np.uint32)


@pytest.mark.parametrize("bits", [1, 2, 3, 4])
def test_ph_is_a_hilbert_curve(oracle, bits):
    g = _grid(bits)
    k = oracle.ph_index(g, bits)
    n = 1 << (3 * bits)
    assert np.array_equal(np.sort(k), np.arange(n, dtype=np.uint64))
    path = g[np.argsort(k)].astype(np.int64)
    assert np.all(np.abs(np.diff(path, axis=0)).sum(1) == 1)   # unit steps
    assert np.array_equal(path[0], [0, 0, 0])
    for level in range(1, bits + 1):
        # the cells of this level: runs of 2^(3 (bits - level)) consecutive indices
        span = 1 << (3 * (bits - level))
        blocks = path.reshape(-1, span, 3) >> (bits - level)
        assert np.all(blocks == blocks[:, :1, :])
        assert len({tuple(b[0]) for b in blocks}) == 1 << (3 * level)
    assert np.array_equal(oracle.ph_coords(k, bits), g)


def test_ph_prefix_decodes_to_the_octant(oracle):
    """The top 3l bits of a 21-bit key are the l-bit key of the octant."""
    rng = np.random.default_rng(91)
    q = rng.integers(0, 1 << 21, size=(2000, 3)).astype(np.uint32)
    k = oracle.ph_index(q, 21)
    for level in (1, 2, 5, 11, 20, 21):
        pre = k >> np.uint64(3 * (21 - level))
        assert np.array_equal(oracle.ph_coords(pre, level), q >> (21 - level))
        assert np.array_equal(oracle.ph_index(q >> (21 - level), level), pre)


def test_ph_keys_of_positions_use_the_morton_quantisation(oracle):
    s = ics.plummer(5000, 92)
    lo, side, scale = oracle.bbox(s.pos)
    km = oracle.morton_keys(s.pos, lo, scale)
    kp = oracle.ph_keys(s.pos, lo, scale)
    # decode both keys to the same 21-bit coordinates
    qm = np.stack([sum((((km >> np.uint64(3 * b + 2 - a)) & np.uint64(1)) << np.uint64(b))
                        for b in range(21)) for a in range(3)], 1).astype(np.uint32)
    assert np.array_equal(oracle.ph_coords(kp, 21), qm)


def _cell_set(tree, q):
    """{(level, octant, count)} of a tree; octant from the quantised
    coordinates q (caller order) of the cell's first particle."""
    c = tree.cells
    first = tree.perm[c["begin"]]
    lev = c["level"].astype(np.int64)
    oct_ = q[first] >> (21 - lev)[:, None].astype(np.uint32)
    return sorted(zip(lev.tolist(), map(tuple, oct_.tolist()), c["count"].tolist()))


@pytest.mark.parametrize("nleaf", [16, 1])
def test_cell_set_identical_under_both_curves(oracle, nleaf):
    s = ics.disk_halo(3000, 9000, 93)
    tm = oracle.build_tree(s.pos, s.mass, nleaf=nleaf)
    tp = oracle.build_tree(s.pos, s.mass, nleaf=nleaf, curve="ph")
    q = oracle.ph_coords(tp.keys, 21)
    assert tm.cells["ncell"] == tp.cells["ncell"]
    assert _cell_set(tm, q) == _cell_set(tp, q)
    # every cell's particles are the same set: the same masses
    mm, mp = tm.mom["M"], tp.mom["M"]
    assert np.allclose(np.sort(mm), np.sort(mp), rtol=1e-12)


def test_ph_tree_forces_match_morton_tree(oracle):
    s = ics.disk_halo(2000, 8000, 94)
    am, pm, _, npc_m = oracle.walk(oracle.build_tree(s.pos, s.mass), 0.5, 0.01)
    tp = oracle.build_tree(s.pos, s.mass, curve="ph")
    ap, pp, _, npc_p = oracle.walk(tp, 0.5, 0.01)
    assert np.allclose(ap, am, rtol=1e-10, atol=1e-12 * np.abs(am).max())
    assert npc_m.sum() == npc_p.sum()
