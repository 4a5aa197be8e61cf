"""Pins of the oracle's group-wise walk (Sec. I.A: opening angle theta;
theta -> 0 reduces the tree-code to direct summation)."""
import numpy as np
import pytest

from workloads import ics


def test_small_theta_is_direct_summation(oracle):
    s = ics.plummer(2048, 7)
    acc, pot, t, npp, npc = oracle.tree_force(s.pos, s.mass, 1e-6, 0.01)
    ad, pd = oracle.direct(s.pos, s.mass, 0.01)
    assert np.all(npc == 0) and np.all(npp == t.n)
    assert np.allclose(acc, ad, rtol=0, atol=1e-12 * np.abs(ad).max())
    assert np.allclose(pot, pd, rtol=1e-12, atol=0)


def test_walk_covers_every_particle_once(oracle):
    s = ics.disk_halo(4000, 16000, 3)
    t = oracle.build_tree(s.pos, s.mass)
    for theta in (0.3, 0.5, 0.7, 1.0):
        _, _, npp, npc, ncov, nself = oracle.walk(t, theta, 0.005, diag=True)
        assert np.all(ncov == t.n)
        assert np.all(nself == 0)
        assert np.all(npp >= t.gcnt)          # the group's own particles


def test_error_falls_with_theta(oracle):
    s = ics.disk_halo(4000, 12000, 5)
    ad, _ = oracle.direct(s.pos, s.mass, 0.005)
    t = oracle.build_tree(s.pos, s.mass)
    med, inter = [], []
    for theta in (0.7, 0.6, 0.5, 0.4, 0.3):
        acc, _, npp, npc = oracle.walk(t, theta, 0.005)
        med.append(np.median(oracle.rel_err(acc, ad)))
        inter.append(((npp + npc) * t.gcnt).sum())
    assert all(med[k + 1] < med[k] for k in range(4)), med
    assert all(inter[k + 1] > inter[k] for k in range(4)), inter
    assert med[-1] < 1e-3


def test_self_potential_excluded_and_zero_softening(oracle):
    # two particles, eps = 0: the walk gives the exact two-body result
    pos = np.array([[0, 0, 0], [1, 0, 0]], np.float32)
    m = np.array([2.0, 3.0], np.float32)
    acc, pot, *_ = oracle.tree_force(pos, m, 0.5, 0.0)
    assert np.allclose(acc, [[3, 0, 0], [-2, 0, 0]]) and np.allclose(pot, [-3, -2])
    # one particle: nothing
    acc, pot, *_ = oracle.tree_force(pos[:1], m[:1], 0.5, 0.1)
    assert np.all(acc == 0) and np.all(pot == 0)


@pytest.mark.parametrize("n", [17, 100, 1000])
def test_small_n_matches_brute_force(oracle, n):
    """Pure-Python brute-force walk for tiny inputs: every group walks the
    tree breadth first with the FP32 opening test and FP64 Eq. (1)-(2)."""
    s = ics.plummer(n, 100 + n)
    t = oracle.build_tree(s.pos, s.mass)
    theta, eps = 0.6, 0.02
    acc, pot, npp, npc = oracle.walk(t, theta, eps)
    c, mo = t.cells, t.mom
    ro = (mo["lf"] / np.float32(theta) + mo["deltaf"]).astype(np.float32)
    ro2 = (ro * ro).astype(np.float32)
    xs = np.stack([t.x, t.y, t.z], 1).astype(np.float64)
    for g in range(t.ngroups):
        gc, gh = t.gc[g], t.gh[g]
        tg = range(t.gbeg[g], t.gbeg[g] + t.gcnt[g])
        a = np.zeros((len(tg), 3))
        p = np.zeros(len(tg))
        q, cpp, cpc = [0], 0, 0
        while q:
            cell = q.pop(0)
            dd = np.maximum(np.abs(mo["comf"][cell] - gc) - gh, np.float32(0)).astype(np.float32)
            d2 = np.float32(np.float32(dd[0] * dd[0] + dd[1] * dd[1]) + dd[2] * dd[2])
            if d2 >= ro2[cell]:
                cpc += 1
                Qv = mo["Q"][cell]
                Qm = np.array([[Qv[0], Qv[3], Qv[4]], [Qv[3], Qv[1], Qv[5]], [Qv[4], Qv[5], Qv[2]]])
                for k, i in enumerate(tg):
                    r = mo["com"][cell] - xs[i]
                    r2 = r @ r + eps * eps
                    ri = r2 ** -0.5
                    Qr = Qm @ r
                    rQr = r @ Qr
                    tr = np.trace(Qm)
                    p[k] += -mo["M"][cell] * ri + 0.5 * tr * ri ** 3 - 1.5 * rQr * ri ** 5
                    a[k] += (mo["M"][cell] * r * ri ** 3 - 1.5 * tr * r * ri ** 5
                             - 3 * Qr * ri ** 5 + 7.5 * rQr * r * ri ** 7)
            elif c["nchild"][cell] == 0:
                cpp += c["count"][cell]
                for j in range(c["begin"][cell], c["begin"][cell] + c["count"][cell]):
                    for k, i in enumerate(tg):
                        r = xs[j] - xs[i]
                        r2 = r @ r + eps * eps
                        a[k] += t.m[j] * r * r2 ** -1.5
                        if j != i:
                            p[k] -= t.m[j] * r2 ** -0.5
            else:
                q.extend(range(c["child0"][cell], c["child0"][cell] + c["nchild"][cell]))
        assert npp[g] == cpp and npc[g] == cpc
        idx = t.perm[list(tg)]
        assert np.allclose(acc[idx], a, rtol=1e-12, atol=1e-14)
        assert np.allclose(pot[idx], p, rtol=1e-12, atol=1e-14)


# --- the opening criterion's geometric guarantee --------------------------------
#
# Every particle y of a cell lies within (sqrt(3)/2) l of the cell's geometric
# centre, so within b = (sqrt(3)/2) l + delta of its centre of mass.  A cell
# accepted for a group (d >= l / theta + delta, d the distance from the
# centre of mass to the group's box) therefore has b / d <= (sqrt(3)/2 l +
# delta) / (l / theta + delta) <= sqrt(3) theta / (1 + sqrt(3) theta / 2)
# (the bound grows with delta <= sqrt(3)/2 l).  The planted variants below
# (delta dropped; the distance measured from the geometric centre) break it
# on cells built for that purpose.

def _bound(theta):
    return np.sqrt(3) * theta / (1 + np.sqrt(3) * theta / 2)


def _worst_ratio(oracle, t, d):
    """max over accepted (group, cell) pairs of max_y |y - com| / dist(com, box)."""
    c = t.cells
    com = t.mom["com"].reshape(-1, 3)
    x = np.stack([t.x, t.y, t.z], 1).astype(np.float64)
    bmax = np.array([np.sqrt(((x[b:b + n] - com[k]) ** 2).sum(1)).max()
                     for k, (b, n) in enumerate(zip(c["begin"], c["count"]))])
    worst = 0.0
    for g in range(t.ngroups):
        cl = d.pc[d.pc_off[g]:d.pc_off[g + 1]]
        if len(cl) == 0:
            continue
        gc, gh = t.gc[g].astype(np.float64), t.gh[g].astype(np.float64)
        gap = np.maximum(np.abs(com[cl] - gc) - gh, 0.0)
        worst = max(worst, float((bmax[cl] / np.sqrt((gap ** 2).sum(1))).max()))
    return worst


def _lopsided_set():
    """A cluster of targets in [0, 1/16)^3 and two level-2 leaves of 16
    particles in [1/2, 1) x [0, 1/4)^2: one with its mass at the corner far
    from the targets (x in [1/2, 3/4)), one at the near corner (x in [3/4, 1))."""
    rng = np.random.default_rng(81)
    tgt = rng.uniform(0, 1 / 16, (200, 3))
    tgt[0] = 0.0
    far = rng.uniform([0.5, 0, 0], [0.75, 0.25, 0.25], (16, 3))
    far[0] = [0.7499, 0.2499, 0.2499]      # the heavy particle
    far[1] = [0.5, 0.0, 0.0]               # a light one at the opposite corner
    near = rng.uniform([0.75, 0, 0], [1.0, 0.25, 0.25], (16, 3))
    near[0] = [0.7501, 0.0001, 0.0001]
    near[1] = [0.9999, 0.2499, 0.2499]
    rest = np.array([[0.9, 0.4, 0.4], [1.0, 0.999, 0.999]])
    pos = np.concatenate([tgt, far, near, rest]).astype(np.float32)
    m = np.concatenate([np.full(200, 1e-3), [1.0], np.full(15, 1e-6), [1.0], np.full(15, 1e-6),
                        [1e-3, 1e-3]]).astype(np.float32)
    return pos, m


def _variant(oracle, t, theta, mutate):
    import copy
    v = copy.copy(t)
    v.mom = dict(t.mom)
    mutate(v)
    return oracle.record_decisions(v, theta)


def _centres(t):
    c = t.cells
    lvl, pre = c["level"].astype(np.int64), c["prefix"].astype(np.uint64)
    q = np.zeros((len(lvl), 3), np.int64)
    for b in range(21):
        for a, sh in ((0, 2), (1, 1), (2, 0)):
            bit = ((pre >> np.uint64(3 * b + sh)) & np.uint64(1)).astype(np.int64)
            q[:, a] |= np.where(b < lvl, bit, 0) << b
    l = np.float64(t.side) * 2.0 ** (-lvl.astype(np.float64))
    return t.lo.astype(np.float64) + (q + 0.5) * l[:, None]


def test_accepted_cells_satisfy_the_opening_bound(oracle):
    pos, m = _lopsided_set()
    t = oracle.build_tree(pos, m)
    # the designed leaves exist: level 2, 16 particles each
    lv, cnt = t.cells["level"], t.cells["count"]
    assert ((lv == 2) & (cnt == 16)).sum() >= 2
    for theta in (0.4, 0.5):
        d = oracle.record_decisions(t, theta)
        assert _worst_ratio(oracle, t, d) <= _bound(theta) * (1 + 1e-5), theta
    s = ics.plummer(4096, 82)
    tp = oracle.build_tree(s.pos, s.mass)
    for theta in (0.3, 0.5, 0.7, 1.0):
        d = oracle.record_decisions(tp, theta)
        assert _worst_ratio(oracle, tp, d) <= _bound(theta) * (1 + 1e-5), theta


def test_planted_opening_mistakes_break_the_bound(oracle):
    """Dropping delta, or measuring the distance from the geometric centre,
    accepts a lopsided leaf that the bound forbids; the oracle opens it."""
    pos, m = _lopsided_set()
    t = oracle.build_tree(pos, m)

    def no_delta(v):
        v.mom["deltaf"] = np.zeros_like(t.mom["deltaf"])

    def from_centre(v):
        v.mom["comf"] = _centres(t).astype(np.float32)

    assert _worst_ratio(oracle, t, _variant(oracle, t, 0.4, no_delta)) > _bound(0.4) * 1.01
    assert _worst_ratio(oracle, t, _variant(oracle, t, 0.5, from_centre)) > _bound(0.5) * 1.01
    # the oracle's own decisions on the same set keep it
    for theta in (0.4, 0.5):
        assert _worst_ratio(oracle, t, oracle.record_decisions(t, theta)) <= _bound(theta) * (1 + 1e-5)
