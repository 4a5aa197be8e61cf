"""CPU oracle for the multi-domain steps of the tree-code (FP64 forces, plain
numpy + C).

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the GPU library or
its binding.  It shares no code with the HIP path.

Steps (paper: Bedorf et al., SC14, arXiv:1412.0659):
  flop-weighted decomposition   Sec. III.B.1 (cut the space-filling curve into
                                p pieces that balance the walk's operations,
                                no piece above a cap on the particle count)
                                with the operation counts of Sec. VI.A (23 per
                                particle-particle and 65 per particle-cell
                                interaction): exact over all keys, and by the
                                paper's two-level sampling
  domain trees                  Sec. III.B.1 (every domain keys its particles
                                in the one global box, so each local tree is a
                                branch of one global octree)
  boundary tree                 Sec. III.B.2 (the local tree cut down to the
                                cells on the edge of the local particle set
                                and their parents)
  local essential tree (LET)    Sec. III.B.2 (the cells and particles of a
                                remote tree that the local targets reach, and
                                whether the remote boundary tree suffices)
  remote walk                   Sec. III.B.2 (forces on the local particles
                                from a remote domain's tree)

Readings of the paper (it gives no formulas for these steps):
  * cost of a particle = 23 npp + 65 npc of its group's last walk;
  * cut j is the first particle where the running cost reaches j/p of the
    total, then clamped so no domain holds more than floor(cap n / p)
    particles (cap = 1.3: at most 30% above the average);
  * boundary cells: descend from the root through cells holding more than
    ncrit particles, stopping at cells of at most ncrit particles, leaves
    and the level L, the deepest at which the boundary tree has at most
    max_cells cells;
  * a domain's target boxes for LET construction are the tight boxes of its
    boundary cells, each side widened by 2^-16 (|lo|_max + side) of the
    global box, so any target group inside a boundary cell opens only cells
    that the cell's box opens, whatever the FP32 rounding.
"""
from __future__ import annotations

import numpy as np

from . import oracle as O

PP_FLOPS = 23
PC_FLOPS = 65


# --- decomposition (Sec. III.B.1) -------------------------------------------------

def particle_cost(n, gbeg, gcnt, npp, npc):
    """Per sorted particle: the walk operations of its group (Sec. VI.A)."""
    cost = np.zeros(n, np.int64)
    w = PP_FLOPS * np.asarray(npp, np.int64) + PC_FLOPS * np.asarray(npc, np.int64)
    for b, c, wg in zip(np.asarray(gbeg, np.int64), np.asarray(gcnt, np.int64), w):
        cost[b:b + c] = wg
    return cost


def decompose(cost, p: int, cap: float):
    """Cuts 0 = c_0 <= c_1 <= ... <= c_p = n of the sorted particles into p
    domains of equal cost, no domain above floor(cap n / p) particles."""
    cost = np.asarray(cost, np.int64)
    n = cost.shape[0]
    C = int(np.floor(float(np.float32(cap)) * n / p))
    if C * p < n:
        raise ValueError("cap * n / p too small to hold n particles")
    S = [0]
    for c in cost.tolist():
        S.append(S[-1] + int(c))
    W = S[-1]
    cuts = [0]
    for j in range(1, p):
        t = n
        for i in range(n + 1):          # first i with S_i >= W j / p
            if S[i] * p >= W * j:
                t = i
                break
        lo = max(cuts[-1], n - (p - j) * C)
        hi = min(cuts[-1] + C, n)
        cuts.append(min(max(t, lo), hi))
    cuts.append(n)
    return np.asarray(cuts, np.int64)


def _samples(keys_local, cost_local, m):
    """m cost-weighted samples of one process's keys (in key order): sample j
    is the key of the particle whose cost interval holds the point
    (j + 1/2) W / m of the process's total cost W."""
    S = 0
    out = []
    W = int(sum(int(c) for c in cost_local))
    j = 0
    for k, c in zip(keys_local.tolist(), cost_local.tolist()):
        S1 = S + int(c)
        while j < m and 2 * m * S1 >= (2 * j + 1) * W:
            out.append(k)
            j += 1
        S = S1
    return out, W


def _equal_weight_cuts(samples, pieces):
    """Boundary keys cutting (key, weight) samples, sorted by key (ties in
    input order), into `pieces` runs of equal total weight: boundary t is the
    key of the first sample at which the weight before it reaches t / pieces
    of the total."""
    order = sorted(range(len(samples)), key=lambda i: samples[i][0])
    T = sum(w for _, w in samples)
    out = []
    S = 0
    t = 1
    for i in order:
        while t < pieces and S * pieces >= T * t:
            out.append(samples[i][0])
            t += 1
        S += samples[i][1]
    while t < pieces:
        out.append(None)   # fewer samples than pieces: an empty piece at the end
        t += 1
    return out


def decompose_sampled(skeys, cost, owner, px, py, m1, m2, cap):
    """The two-level sampling cut (Sec. III.B.1) emulated in one process.
    skeys: sorted keys, cost: cost of each sorted particle, owner: the process
    (0 .. px py - 1) holding it.  Level 1: every process draws m1 cost-weighted
    samples of its keys, each carrying its total cost W_q; one DD process cuts
    them into px equal-weight pieces.  Level 2: every process draws m2
    samples, each goes to the piece its key falls in, and each piece's DD
    process cuts its samples into py pieces.  The p - 1 boundary keys give
    the domains [B_d, B_{d+1}); the slots are clamped by the particle cap of
    `decompose`.  Returns (cuts [p + 1], boundary keys [p - 1])."""
    skeys = np.asarray(skeys, np.uint64)
    cost = np.asarray(cost, np.int64)
    owner = np.asarray(owner, np.int64)
    n = skeys.shape[0]
    p = px * py
    C = int(np.floor(float(np.float32(cap)) * n / p))
    if C * p < n:
        raise ValueError("cap * n / p too small to hold n particles")
    local = [np.nonzero(owner == q)[0] for q in range(p)]   # key order kept
    s1 = []
    for q in range(p):
        ks, W = _samples(skeys[local[q]], cost[local[q]], m1)
        s1 += [(k, W) for k in ks]
    b1 = _equal_weight_cuts(s1, px)
    top = [k for k in b1 if k is not None]
    buckets = [[] for _ in range(px)]
    for q in range(p):
        ks, W = _samples(skeys[local[q]], cost[local[q]], m2)
        for k in ks:
            t = sum(1 for b in top if b <= k)   # the piece whose key range holds k
            buckets[t].append((k, W))
    # a missing boundary (fewer samples than pieces) closes its piece at the
    # end of the enclosing range: the next top boundary, else past every key
    big = int(np.iinfo(np.uint64).max)
    tops = [big if b is None else int(b) for b in b1]
    bk = []
    for t in range(px):
        if t > 0:
            bk.append(tops[t - 1])
        end = tops[t] if t < px - 1 else big
        bk += [end if b is None else int(b) for b in _equal_weight_cuts(buckets[t], py)]
    cuts = [0]
    for j in range(1, p):
        t = int(np.searchsorted(skeys, np.uint64(bk[j - 1]), side="left"))
        lo = max(cuts[-1], n - (p - j) * C)
        hi = min(cuts[-1] + C, n)
        cuts.append(min(max(t, lo), hi))
    cuts.append(n)
    return np.asarray(cuts, np.int64), np.asarray(bk, np.uint64)


# --- boundary tree (Sec. III.B.2) -------------------------------------------------

def boundary(tree: O.Tree, max_cells: int, ncrit: int = O.NCRIT):
    """The boundary tree of a domain tree: (L, in_boundary, terminal) with
    flags per cell; terminal cells partition the particles."""
    c = tree.cells
    nc = c["ncell"]
    count, nchild, parent, level = c["count"], c["nchild"], c["parent"], c["level"]
    inb = np.zeros(nc, bool)
    inb[0] = True
    for i in range(1, nc):
        inb[i] = count[parent[i]] > ncrit
    per_level = np.bincount(level[inb], minlength=O.NLEVELS)
    tot, L = 0, -1
    for lev in range(O.NLEVELS):
        if tot + per_level[lev] > max_cells:
            break
        tot += per_level[lev]
        L = lev
    if L < 0:
        raise ValueError("max_cells < 1")
    inb &= level <= L
    small = (count <= ncrit) | (nchild == 0)
    term = inb & ((level == L) | small)
    return L, inb, term


def margin(box):
    """Widening of the target boxes: fl32(2^-16 (max |lo| + side))."""
    lo, side = box
    lo = np.asarray(lo, np.float32)
    r = np.float32(np.float32(np.max(np.abs(lo))) + np.float32(side))
    return np.float32(r * np.float32(2.0 ** -16))


def boundary_boxes(tree: O.Tree, term, box):
    """Tight FP32 boxes of the terminal boundary cells, in cell order:
    centre (min + max) / 2, half size (max - min) / 2 + margin."""
    c = tree.cells
    ids = np.nonzero(term)[0]
    m = margin(box)
    bc = np.empty((ids.shape[0], 3), np.float32)
    bh = np.empty((ids.shape[0], 3), np.float32)
    xs = (tree.x, tree.y, tree.z)
    for k, i in enumerate(ids):
        b, e = c["begin"][i], c["begin"][i] + c["count"][i]
        for a in range(3):
            mn = np.float32(xs[a][b:e].min())
            mx = np.float32(xs[a][b:e].max())
            bc[k, a] = np.float32((mn + mx) * np.float32(0.5))
            bh[k, a] = np.float32(np.float32((mx - mn) * np.float32(0.5)) + m)
    return ids, bc, bh


# --- local essential tree (Sec. III.B.2) -----------------------------------------

def let_mark(src: O.Tree, theta: float, bc, bh, bterm=None):
    """(visited, opened, insufficient) over the source tree's cells for the
    target boxes bc, bh; insufficient: an opened cell is terminal in the
    source's boundary tree (flags bterm)."""
    c = src.cells
    nc = c["ncell"]
    ro2 = O.open_radius2(src.mom["lf"], src.mom["deltaf"], theta)
    vis = np.zeros(nc, np.uint8)
    opn = np.zeros(nc, np.uint8)
    bt = None
    if bterm is not None:
        bt = np.ascontiguousarray(bterm, dtype=np.uint8)
    ins = O.lib().orc_let_mark(
        bc.shape[0], np.ascontiguousarray(bc, np.float32).reshape(-1),
        np.ascontiguousarray(bh, np.float32).reshape(-1), nc, c["child0"], c["nchild"],
        O._f32(src.mom["comf"].reshape(-1)), ro2,
        None if bt is None else bt.ctypes.data, vis, opn)
    return vis.astype(bool), opn.astype(bool), bool(ins)


def prune(src: O.Tree, keep, expand):
    """The source tree with only the kept cells: an expanded cell keeps its
    children (internal) or particles (leaf); any other kept cell becomes a
    leaf with no particles.  Returns cell arrays in the source's numbering
    (dropped cells unreachable) for the remote walk."""
    c = src.cells
    count = np.where(keep & expand, c["count"], 0).astype(np.int64)
    nchild = np.where(keep & expand, c["nchild"], 0).astype(np.int32)
    return dict(c, count=count, nchild=nchild)


# --- remote walk (Sec. III.B.2) ---------------------------------------------------

def walk_remote(tgt: O.Tree, src: O.Tree, theta: float, eps: float, cells=None, groups=None):
    """Forces on tgt's particles (caller order of tgt; NaN outside the listed
    groups) from src's tree, and per-group (npp, npc) of tgt's groups (-1
    where not walked).  cells replaces src's topology (count, nchild) by a
    pruned one; moments stay src's.  groups: tgt's groups to walk (all by
    default)."""
    c = src.cells if cells is None else cells
    n = tgt.n
    ro2 = O.open_radius2(src.mom["lf"], src.mom["deltaf"], theta)
    glist = np.arange(tgt.ngroups, dtype=np.int64) if groups is None else \
        np.ascontiguousarray(np.unique(groups), dtype=np.int64)
    acc_s = np.full(3 * n, np.nan)
    pot_s = np.full(n, np.nan)
    npp = np.full(tgt.ngroups, -1, np.int64)
    npc = np.full(tgt.ngroups, -1, np.int64)
    ncov = np.full(tgt.ngroups, -1, np.int64)
    O.lib().orc_walk_remote(
        glist.shape[0], glist, tgt.gbeg, tgt.gcnt, O._f32(tgt.gc.reshape(-1)),
        O._f32(tgt.gh.reshape(-1)), tgt.x, tgt.y, tgt.z, src.cells["ncell"],
        np.ascontiguousarray(c["begin"], np.int64), np.ascontiguousarray(c["count"], np.int64),
        np.ascontiguousarray(c["child0"], np.int64), np.ascontiguousarray(c["nchild"], np.int32),
        src.mom["M"], O._f64(src.mom["com"].reshape(-1)), O._f64(src.mom["Q"].reshape(-1)),
        O._f32(src.mom["comf"].reshape(-1)), ro2, src.x, src.y, src.z, src.m, float(eps),
        acc_s, pot_s, npp, npc, ncov)
    acc = np.full((n, 3), np.nan)
    pot = np.full(n, np.nan)
    acc[tgt.perm] = acc_s.reshape(n, 3)
    pot[tgt.perm] = pot_s
    return acc, pot, npp, npc, ncov


def domain_forces(pos, mass, cuts_perm, box, theta, eps, curve="morton"):
    """Forces on every particle (caller order) when the particles are split
    into the domains given as lists of caller indices: each domain's own
    tree walk plus the walks of every other domain's tree."""
    pos = np.asarray(pos, np.float32).reshape(-1, 3)
    mass = np.asarray(mass, np.float32).reshape(-1)
    trees = [O.build_tree(pos[ix], mass[ix], curve=curve, box=box) for ix in cuts_perm]
    acc = np.zeros((pos.shape[0], 3))
    pot = np.zeros(pos.shape[0])
    for d, ix in enumerate(cuts_perm):
        a, p, _, _ = O.walk(trees[d], theta, eps)
        for e in range(len(cuts_perm)):
            if e != d:
                ar, pr, _, _, _ = walk_remote(trees[d], trees[e], theta, eps)
                a = a + ar
                p = p + pr
        acc[ix] = a
        pot[ix] = p
    return acc, pot, trees
