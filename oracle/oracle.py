"""CPU oracle for the Barnes-Hut tree-code hot path (FP64, plain C + numpy).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library or its binding.  It
shares no code with the HIP path.

Steps (paper: Bedorf et al., SC14, arXiv:1412.0659):
  bounding box + Morton keys    Sec. III.B.1 (space-filling-curve keys from
                                the bounding box; Morton in place of
                                Peano-Hilbert, the same octree cell set)
  stable key sort               Table II "Sorting SFC" (numpy stable argsort)
  octree build                  Sec. I.A (split octants until a cell holds at
                                most 16 particles)
  groups                        target groups of the group-wise walk
  moments                       Sec. VI.A Eq. (1): mass, centre of mass and
                                the 3x3 quadrupole
  walk + forces                 Sec. I.A opening angle theta; Sec. VI.A
                                Eq. (1)-(2); Plummer softening (Sec. IV)
  direct summation              the theta -> 0 limit of Sec. I.A
  leapfrog (KDK)                Sec. III.B.2 (second-order leap-frog)
  differentiation form          not in the paper: the walk's decisions are
                                recorded and frozen, the forces replayed in
                                FP64 and differentiated by a hand-written
                                reverse sweep (force VJP, KDK transpose)
  surface density               the face-on surface density the paper shows
                                for its Milky Way run (Sec. IV), as bilinear
                                cloud-in-cell on a polar grid
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from .build import ensure_built

NLEAF = 16
NCRIT = 64
NLEVELS = 22

_lib = None

_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
_i64 = ctypes.c_int64
_int = ctypes.c_int


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(ensure_built())
        L.orc_num_threads.restype = _int
        L.orc_bbox.argtypes = [_i64, _f32p, _f32p, _f32p, _f32p]
        L.orc_keys.argtypes = [_i64, _f32p, _f32p, ctypes.c_float, _u64p]
        L.orc_build.argtypes = [_i64, _u64p, _int, _i64, _i32p, _u64p, _i64p, _i64p, _i64p,
                                _i32p, _i64p, _i64p]
        L.orc_build.restype = _i64
        L.orc_groups.argtypes = [_i64, _i64p, _i64p, _i32p, _i64p, _int, _i64p, _i64p, _i64p]
        L.orc_groups.restype = _i64
        L.orc_group_boxes.argtypes = [_i64, _i64p, _i64p, _f32p, _f32p, _f32p, _f32p, _f32p]
        L.orc_moments.argtypes = [_i64, _i32p, _u64p, _i64p, _i64p, _i64p, _i32p, _f32p, _f32p,
                                  _f32p, _f32p, _f32p, ctypes.c_float, _int, _f64p, _f64p, _f64p,
                                  _f64p, _f32p, _f32p, _f32p]
        _u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        L.orc_ph_index.argtypes = [_i64, _u32p, _int, _u64p]
        L.orc_ph_coords.argtypes = [_i64, _u64p, _int, _u32p]
        L.orc_keys_ph.argtypes = [_i64, _f32p, _f32p, ctypes.c_float, _u64p]
        L.orc_open_radius.argtypes = [_i64, _f32p, _f32p, ctypes.c_float, _f32p]
        L.orc_walk.argtypes = [_i64, _i64p, _i64p, _i64p, _f32p, _f32p, _i64, _i64p, _i64p,
                               _i64p, _i32p, _f64p, _f64p, _f64p, _f32p, _f32p, _f32p, _f32p,
                               _f32p, _f32p, ctypes.c_double, _f64p, _f64p, _i64p, _i64p,
                               _i64p, _i64p]
        L.orc_direct.argtypes = [_i64, _f64p, _f64p, _i64, _i64p, ctypes.c_double, _f64p, _f64p]
        L.orc_expansion.argtypes = [_i64, _f64p, ctypes.c_double, _f64p, _f64p, ctypes.c_double,
                                    _f64p, _f64p]
        L.orc_walk_remote.argtypes = [_i64, _i64p, _i64p, _i64p, _f32p, _f32p, _f32p, _f32p,
                                      _f32p, _i64, _i64p, _i64p, _i64p, _i32p, _f64p, _f64p,
                                      _f64p, _f32p, _f32p, _f32p, _f32p, _f32p, _f32p,
                                      ctypes.c_double, _f64p, _f64p, _i64p, _i64p, _i64p]
        _u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
        L.orc_let_mark.argtypes = [_i64, _f32p, _f32p, _i64, _i64p, _i32p, _f32p, _f32p,
                                   ctypes.c_void_p, _u8p, _u8p]
        L.orc_let_mark.restype = _int
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().orc_num_threads())


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --- O1/O2/O3 ----------------------------------------------------------------

def bbox(pos):
    pos = _f32(pos).reshape(-1, 3)
    lo = np.zeros(3, np.float32)
    side = np.zeros(1, np.float32)
    scale = np.zeros(1, np.float32)
    lib().orc_bbox(pos.shape[0], pos, lo, side, scale)
    return lo, np.float32(side[0]), np.float32(scale[0])


def morton_keys(pos, lo, scale):
    pos = _f32(pos).reshape(-1, 3)
    out = np.empty(pos.shape[0], np.uint64)
    lib().orc_keys(pos.shape[0], pos, _f32(lo), ctypes.c_float(scale), out)
    return out


def ph_keys(pos, lo, scale):
    """63-bit Peano-Hilbert keys with the Morton key's quantisation."""
    pos = _f32(pos).reshape(-1, 3)
    out = np.empty(pos.shape[0], np.uint64)
    lib().orc_keys_ph(pos.shape[0], pos, _f32(lo), ctypes.c_float(scale), out)
    return out


def ph_index(q, bits):
    """Peano-Hilbert index of integer points q [n, 3] with `bits` per axis."""
    q = np.ascontiguousarray(q, dtype=np.uint32).reshape(-1, 3)
    out = np.empty(q.shape[0], np.uint64)
    lib().orc_ph_index(q.shape[0], q, int(bits), out)
    return out


def ph_coords(keys, bits):
    """Inverse of ph_index."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    out = np.empty((keys.shape[0], 3), np.uint32)
    lib().orc_ph_coords(keys.shape[0], keys, int(bits), out)
    return out


def sort_keys(keys):
    """Stable ascending sort; equal keys keep their input order."""
    return np.argsort(keys, kind="stable")


# --- O4/O5 ---------------------------------------------------------------------

def cell_capacity(n: int, nleaf: int = NLEAF) -> int:
    """Upper bound on the cell count: at most n leaves (disjoint, non-empty)
    plus, on each of the 21 levels that can hold internal cells, at most
    n // (nleaf + 1) disjoint cells holding more than nleaf particles."""
    return n + 21 * (n // (nleaf + 1)) + 1


def build_cells(skeys, nleaf: int = NLEAF):
    skeys = np.ascontiguousarray(skeys, dtype=np.uint64)
    n = skeys.shape[0]
    cap = cell_capacity(n, nleaf)
    level = np.empty(cap, np.int32)
    prefix = np.empty(cap, np.uint64)
    begin = np.empty(cap, np.int64)
    count = np.empty(cap, np.int64)
    child0 = np.empty(cap, np.int64)
    nchild = np.empty(cap, np.int32)
    parent = np.empty(cap, np.int64)
    ls = np.zeros(NLEVELS + 1, np.int64)
    nc = lib().orc_build(n, skeys, nleaf, cap, level, prefix, begin, count, child0, nchild,
                         parent, ls)
    if nc < 0:
        raise RuntimeError("cell capacity exceeded")
    return dict(level=level[:nc].copy(), prefix=prefix[:nc].copy(), begin=begin[:nc].copy(),
                count=count[:nc].copy(), child0=child0[:nc].copy(), nchild=nchild[:nc].copy(),
                parent=parent[:nc].copy(), level_start=ls, ncell=int(nc))


def make_groups(cells, ncrit: int = NCRIT):
    nc = cells["ncell"]
    n = int(cells["count"][0])
    gbeg = np.empty(n, np.int64)
    gcnt = np.empty(n, np.int64)
    gcell = np.empty(n, np.int64)
    ng = lib().orc_groups(nc, cells["begin"], cells["count"], cells["nchild"], cells["parent"],
                          ncrit, gbeg, gcnt, gcell)
    return gbeg[:ng].copy(), gcnt[:ng].copy(), gcell[:ng].copy()


def group_boxes(gbeg, gcnt, x, y, z):
    ng = gbeg.shape[0]
    gc = np.empty(3 * ng, np.float32)
    gh = np.empty(3 * ng, np.float32)
    lib().orc_group_boxes(ng, gbeg, gcnt, _f32(x), _f32(y), _f32(z), gc, gh)
    return gc.reshape(ng, 3), gh.reshape(ng, 3)


# --- O6 --------------------------------------------------------------------------

def moments(cells, x, y, z, m, lo, side, curve="morton"):
    nc = cells["ncell"]
    M = np.empty(nc)
    S = np.empty(3 * nc)
    com = np.empty(3 * nc)
    Q = np.empty(6 * nc)
    comf = np.empty(3 * nc, np.float32)
    lf = np.empty(nc, np.float32)
    deltaf = np.empty(nc, np.float32)
    lib().orc_moments(nc, cells["level"], cells["prefix"], cells["begin"], cells["count"],
                      cells["child0"], cells["nchild"], _f32(x), _f32(y), _f32(z), _f32(m),
                      _f32(lo), ctypes.c_float(side), 1 if curve == "ph" else 0, M, S, com, Q,
                      comf, lf, deltaf)
    return dict(M=M, S=S.reshape(nc, 3), com=com.reshape(nc, 3), Q=Q.reshape(nc, 6),
                comf=comf.reshape(nc, 3), lf=lf, deltaf=deltaf)


def open_radius2(lf, deltaf, theta):
    out = np.empty(lf.shape[0], np.float32)
    lib().orc_open_radius(lf.shape[0], _f32(lf), _f32(deltaf), ctypes.c_float(theta), out)
    return out


# --- the whole tree ------------------------------------------------------------

@dataclass
class Tree:
    n: int
    lo: np.ndarray
    side: np.float32
    scale: np.float32
    keys: np.ndarray       # caller order
    perm: np.ndarray       # sorted slot -> caller index
    skeys: np.ndarray
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    m: np.ndarray
    cells: dict
    gbeg: np.ndarray
    gcnt: np.ndarray
    gcell: np.ndarray
    gc: np.ndarray
    gh: np.ndarray
    mom: dict

    @property
    def ngroups(self):
        return int(self.gbeg.shape[0])

    def group_of_sorted(self):
        g = np.zeros(self.n, np.int64)
        g[self.gbeg[1:]] = 1
        return np.cumsum(g)


def fixed_box(lo, side):
    """A caller-given key box (Sec. III.B.1: every domain maps its particles
    to keys with the one global box): lo, side, fl32(2^21 / side)."""
    lo = np.ascontiguousarray(lo, dtype=np.float32).reshape(3)
    side = np.float32(side)
    return lo, side, np.float32(2097152.0 / float(side))


def build_tree(pos, mass, nleaf: int = NLEAF, ncrit: int = NCRIT, curve: str = "morton",
               box=None) -> Tree:
    """The whole tree of Sec. III.B.1 / Sec. I.A; curve "morton" or "ph"
    (Peano-Hilbert, the paper's curve): the same cells in another order.
    box = (lo[3], side) keys the particles in that box instead of their own
    bounding box (a coordinate below lo takes the first cell, one at or past
    lo + side the last)."""
    pos = _f32(pos).reshape(-1, 3)
    mass = _f32(mass).reshape(-1)
    n = pos.shape[0]
    lo, side, scale = bbox(pos) if box is None else fixed_box(*box)
    keys = ph_keys(pos, lo, scale) if curve == "ph" else morton_keys(pos, lo, scale)
    perm = sort_keys(keys)
    skeys = keys[perm]
    sp = pos[perm]
    x, y, z = (np.ascontiguousarray(sp[:, a]) for a in range(3))
    m = np.ascontiguousarray(mass[perm])
    cells = build_cells(skeys, nleaf)
    gbeg, gcnt, gcell = make_groups(cells, ncrit)
    gc, gh = group_boxes(gbeg, gcnt, x, y, z)
    mom = moments(cells, x, y, z, m, lo, side, curve)
    return Tree(n, lo, side, scale, keys, perm, skeys, x, y, z, m, cells, gbeg, gcnt, gcell,
                gc, gh, mom)


def walk(tree: Tree, theta: float, eps: float, groups=None, diag=False):
    """Tree forces for the targets of the listed groups (all groups by default).

    Returns (acc[N,3], pot[N]) in caller order (NaN where not computed) and
    per-group (npp, npc) counts (-1 where not walked).  With ``diag`` also
    returns per-group (ncov, nself): particles covered by the interaction
    lists and accepted cells holding a particle of the group."""
    n = tree.n
    ro2 = open_radius2(tree.mom["lf"], tree.mom["deltaf"], theta)
    glist = np.arange(tree.ngroups, dtype=np.int64) if groups is None else \
        np.ascontiguousarray(np.unique(groups), dtype=np.int64)
    acc_s = np.full(3 * n, np.nan)
    pot_s = np.full(n, np.nan)
    npp = np.full(tree.ngroups, -1, np.int64)
    npc = np.full(tree.ngroups, -1, np.int64)
    ncov = np.full(tree.ngroups, -1, np.int64)
    nself = np.full(tree.ngroups, -1, np.int64)
    c = tree.cells
    lib().orc_walk(glist.shape[0], glist, tree.gbeg, tree.gcnt, _f32(tree.gc.reshape(-1)),
                   _f32(tree.gh.reshape(-1)), c["ncell"], c["begin"], c["count"], c["child0"],
                   c["nchild"], tree.mom["M"], _f64(tree.mom["com"].reshape(-1)),
                   _f64(tree.mom["Q"].reshape(-1)), _f32(tree.mom["comf"].reshape(-1)), ro2,
                   tree.x, tree.y, tree.z, tree.m, float(eps), acc_s, pot_s, npp, npc, ncov,
                   nself)
    acc = np.full((n, 3), np.nan)
    pot = np.full(n, np.nan)
    acc[tree.perm] = acc_s.reshape(n, 3)
    pot[tree.perm] = pot_s
    if diag:
        return acc, pot, npp, npc, ncov, nself
    return acc, pot, npp, npc


def tree_force(pos, mass, theta, eps, nleaf=NLEAF, ncrit=NCRIT):
    t = build_tree(pos, mass, nleaf, ncrit)
    acc, pot, npp, npc = walk(t, theta, eps)
    return acc, pot, t, npp, npc


def direct(pos, mass, eps, targets=None):
    """Direct-summation accelerations and potentials (FP64) at the targets."""
    pos = _f64(pos).reshape(-1, 3)
    mass = _f64(mass).reshape(-1)
    n = pos.shape[0]
    tgt = np.arange(n, dtype=np.int64) if targets is None else \
        np.ascontiguousarray(targets, dtype=np.int64)
    acc = np.empty(3 * tgt.shape[0])
    pot = np.empty(tgt.shape[0])
    lib().orc_direct(n, pos.reshape(-1), mass, tgt.shape[0], tgt, float(eps), acc, pot)
    return acc.reshape(-1, 3), pot


def expansion(targets, mc, comc, qc, eps=0.0):
    """Eq. (1)/(2) of a single cell (mass, centre, quadrupole xx,yy,zz,xy,xz,yz)."""
    t = _f64(targets).reshape(-1, 3)
    acc = np.empty(3 * t.shape[0])
    pot = np.empty(t.shape[0])
    lib().orc_expansion(t.shape[0], t.reshape(-1), float(mc), _f64(comc), _f64(qc), float(eps),
                        acc, pot)
    return acc.reshape(-1, 3), pot


# --- O10: second-order leapfrog (kick-drift-kick) --------------------------------

def leapfrog(pos, vel, mass, dt, steps, force):
    """KDK leapfrog in FP64 with a shared time step.

    ``force(pos64) -> acc64`` gives the accelerations; the force at the
    initial positions is computed first.  Returns (pos, vel) after ``steps``.
    """
    x = _f64(pos).reshape(-1, 3).copy()
    v = _f64(vel).reshape(-1, 3).copy()
    a = force(x)
    for _ in range(steps):
        v = v + 0.5 * dt * a
        x = x + dt * v
        a = force(x)
        v = v + 0.5 * dt * a
    return x, v


def direct_force_fn(mass, eps):
    return lambda x: direct(x, mass, eps)[0]


def tree_force_fn(mass, theta, eps):
    """Tree force on positions rounded to FP32 (the tree is defined on FP32)."""
    return lambda x: tree_force(x.astype(np.float32), mass, theta, eps)[0]


def rel_err(a, ref):
    """Per-target relative error of vectors ||a - ref|| / ||ref||."""
    a = np.asarray(a, np.float64)
    ref = np.asarray(ref, np.float64)
    if a.ndim == 1:
        return np.abs(a - ref) / np.abs(ref)
    return np.sqrt(((a - ref) ** 2).sum(1)) / np.sqrt((ref ** 2).sum(1))


# --- differentiation with frozen decisions ------------------------------------

def _declare_adjoint(L):
    if getattr(L, "_adjoint_declared", False):
        return
    L.orc_walk_record.argtypes = [_i64, _i64p, _i64p, _f32p, _f32p, _i64, _i64p, _i32p, _f32p,
                                  _f32p, _i64p, ctypes.c_void_p, _i64p, ctypes.c_void_p]
    L.orc_replay.argtypes = [_i64, _i64p, _i64p, _i64, _i64p, _i64p, _i64p, _i32p, _i64p, _i64p,
                             _i64p, _i64p, _f64p, _f64p, ctypes.c_double, _f64p, _f64p, _f64p,
                             _f64p, _f64p]
    L.orc_replay_vjp.argtypes = [_i64, _i64p, _i64p, _i64, _i64p, _i64p, _i64p, _i32p, _i64p,
                                 _i64p, _i64p, _i64p, _f64p, _f64p, ctypes.c_double, _f64p, _f64p,
                                 _f64p, _f64p, _f64p, _f64p, _f64p, _f64p, _f64p]
    L._adjoint_declared = True


@dataclass
class Decisions:
    """The walk's decisions for every group, held fixed for differentiation:
    accepted cells pc[pc_off[g]:pc_off[g+1]] and opened leaves
    lf[lf_off[g]:lf_off[g+1]], on the tree's topology."""
    tree: Tree
    pc_off: np.ndarray
    pc: np.ndarray
    lf_off: np.ndarray
    lf: np.ndarray


def record_decisions(tree: Tree, theta: float) -> Decisions:
    L = lib()
    _declare_adjoint(L)
    c = tree.cells
    ng = tree.ngroups
    ro2 = open_radius2(tree.mom["lf"], tree.mom["deltaf"], theta)
    args = (ng, tree.gbeg, tree.gcnt, _f32(tree.gc.reshape(-1)), _f32(tree.gh.reshape(-1)),
            c["ncell"], c["child0"], c["nchild"], _f32(tree.mom["comf"].reshape(-1)), ro2)
    pc_off = np.zeros(ng + 1, np.int64)
    lf_off = np.zeros(ng + 1, np.int64)
    L.orc_walk_record(*args, pc_off, None, lf_off, None)
    pc = np.zeros(max(int(pc_off[-1]), 1), np.int64)
    lf = np.zeros(max(int(lf_off[-1]), 1), np.int64)
    L.orc_walk_record(*args, pc_off, pc.ctypes.data_as(ctypes.c_void_p), lf_off,
                      lf.ctypes.data_as(ctypes.c_void_p))
    return Decisions(tree, pc_off, pc, lf_off, lf)


def _topo(d: Decisions):
    t = d.tree
    c = t.cells
    return (t.ngroups, t.gbeg, t.gcnt, c["ncell"], c["begin"], c["count"], c["child0"],
            c["nchild"], d.pc_off, d.pc, d.lf_off, d.lf)


def replay(d: Decisions, x_sorted, m_sorted, eps):
    """Force with frozen decisions at FP64 positions/masses in sorted order.
    Returns (acc[N,3], pot[N], M, com, Q) in sorted order."""
    L = lib()
    _declare_adjoint(L)
    nc = d.tree.cells["ncell"]
    n = d.tree.n
    M, com, Q = np.empty(nc), np.empty(3 * nc), np.empty(6 * nc)
    acc, pot = np.empty(3 * n), np.empty(n)
    L.orc_replay(*_topo(d), _f64(x_sorted).reshape(-1), _f64(m_sorted), float(eps), M, com, Q,
                 acc, pot)
    return acc.reshape(n, 3), pot, M, com, Q


def replay_vjp(d: Decisions, x_sorted, m_sorted, eps, u_sorted):
    """u^T d(acc)/d(x, m) for the frozen-decision force (sorted order)."""
    L = lib()
    _declare_adjoint(L)
    x = _f64(x_sorted).reshape(-1)
    m = _f64(m_sorted)
    _, _, M, com, Q = replay(d, x_sorted, m_sorted, eps)
    nc = d.tree.cells["ncell"]
    n = d.tree.n
    lM, lcom, lQ = np.empty(nc), np.empty(3 * nc), np.empty(6 * nc)
    gx, gm = np.zeros(3 * n), np.zeros(n)
    L.orc_replay_vjp(*_topo(d), x, m, float(eps), M, com, Q, _f64(u_sorted).reshape(-1), lM, lcom,
                     lQ, gx, gm)
    return gx.reshape(n, 3), gm


def frozen_force(d: Decisions, x, m, eps):
    """Frozen-decision accelerations at FP64 caller-order positions x."""
    perm = d.tree.perm
    a_s = replay(d, np.asarray(x, np.float64)[perm], np.asarray(m, np.float64)[perm], eps)[0]
    a = np.empty_like(a_s)
    a[perm] = a_s
    return a


def frozen_force_vjp(d: Decisions, x, m, eps, u):
    """u^T d(acc)/d(x, m) of frozen_force (caller order)."""
    perm = d.tree.perm
    gx_s, gm_s = replay_vjp(d, np.asarray(x, np.float64)[perm], np.asarray(m, np.float64)[perm],
                            eps, np.asarray(u, np.float64)[perm])
    gx = np.empty_like(gx_s)
    gm = np.empty_like(gm_s)
    gx[perm] = gx_s
    gm[perm] = gm_s
    return gx, gm


def trajectory_decisions(positions, mass, theta, nleaf=NLEAF, ncrit=NCRIT):
    """Decisions of the walk at each stored step (positions: list of FP32
    [N,3] arrays, caller order): the trees are built from exactly those
    FP32 positions."""
    return [record_decisions(build_tree(p, mass, nleaf, ncrit), theta) for p in positions]


def leapfrog_frozen(x0, v0, m, dt, decs, eps):
    """K = len(decs) - 1 kick-drift-kick steps in FP64, the force at step n
    taken with the frozen decisions decs[n].  Returns (x_K, v_K, [x_n])."""
    h = 0.5 * dt
    x = np.asarray(x0, np.float64).copy()
    v = np.asarray(v0, np.float64).copy()
    xs = [x.copy()]
    a = frozen_force(decs[0], x, m, eps)
    for n in range(len(decs) - 1):
        v = v + h * a
        x = x + dt * v
        xs.append(x.copy())
        a = frozen_force(decs[n + 1], x, m, eps)
        v = v + h * a
    return x, v, xs


def leapfrog_frozen_vjp(x0, v0, m, dt, decs, eps, gxK, gvK):
    """Reverse sweep of leapfrog_frozen: cotangents of (x_K, v_K) ->
    gradients with respect to (x_0, v_0, m).  The two kicks that meet at an
    interior position share the cotangent, so each x_n takes one VJP with
    weight dt (dt/2 at n = 0 and n = K)."""
    h = 0.5 * dt
    K = len(decs) - 1
    _, _, xs = leapfrog_frozen(x0, v0, m, dt, decs, eps)
    gx = np.asarray(gxK, np.float64).copy()
    gv = np.asarray(gvK, np.float64).copy()
    gm = np.zeros(len(m))
    g1, gm1 = frozen_force_vjp(decs[K], xs[K], m, eps, gv)
    gx += h * g1
    gm += h * gm1
    for j in reversed(range(K)):
        gv = gv + dt * gx
        c = dt if j > 0 else h
        g1, gm1 = frozen_force_vjp(decs[j], xs[j], m, eps, gv)
        gx += c * g1
        gm += c * gm1
    return gx, gv, gm


# --- surface density observable (cloud-in-cell on a polar grid) ---------------

def cic_density(pos, mass, sel, grid):
    """Face-on surface density of the selected particles on the polar grid
    (r_min, r_max, n_r, n_phi): cell centres R_i = r_min + (i + 1/2) dR,
    phi_j = (j + 1/2) dphi; bilinear cloud-in-cell weights in (R, phi),
    phi periodic, cells outside [0, n_r) dropped; particles with R outside
    [r_min, r_max) dropped (the inner cut keeps d(phi)/dx ~ 1/R bounded);
    mass / cell area.  FP64."""
    r0, r1, nr, nphi = grid
    pos = np.asarray(pos, np.float64)
    m = np.asarray(mass, np.float64)
    if sel is not None:
        pos, m = pos[sel], m[sel]
    R = np.hypot(pos[:, 0], pos[:, 1])
    keep = (R >= r0) & (R < r1)
    pos, m = pos[keep], m[keep]
    dr = (r1 - r0) / nr
    dphi = 2 * np.pi / nphi
    R = np.hypot(pos[:, 0], pos[:, 1])
    phi = np.mod(np.arctan2(pos[:, 1], pos[:, 0]), 2 * np.pi)
    u = (R - r0) / dr - 0.5
    v = phi / dphi - 0.5
    i0 = np.floor(u).astype(np.int64)
    j0 = np.floor(v).astype(np.int64)
    fu, fv = u - i0, v - j0
    acc = np.zeros((nr, nphi))
    for a in (0, 1):
        for b in (0, 1):
            w = (fu if a else 1 - fu) * (fv if b else 1 - fv) * m
            i = i0 + a
            j = np.mod(j0 + b, nphi)
            ok = (i >= 0) & (i < nr)
            np.add.at(acc, (i[ok], j[ok]), w[ok])
    redge = r0 + dr * np.arange(nr + 1)
    area = 0.5 * dphi * (redge[1:] ** 2 - redge[:-1] ** 2)
    return acc / area[:, None]


def cic_density_vjp(pos, mass, sel, grid, g):
    """Gradient of sum(g * cic_density) with respect to pos and mass."""
    r0, r1, nr, nphi = grid
    pos = np.asarray(pos, np.float64)
    m_all = np.asarray(mass, np.float64)
    idx = np.arange(len(m_all)) if sel is None else np.nonzero(sel)[0]
    Rall = np.hypot(pos[idx, 0], pos[idx, 1])
    idx = idx[(Rall >= r0) & (Rall < r1)]
    p, m = pos[idx], m_all[idx]
    dr = (r1 - r0) / nr
    dphi = 2 * np.pi / nphi
    x, y = p[:, 0], p[:, 1]
    R = np.hypot(x, y)
    phi = np.mod(np.arctan2(y, x), 2 * np.pi)
    u = (R - r0) / dr - 0.5
    v = phi / dphi - 0.5
    i0 = np.floor(u).astype(np.int64)
    j0 = np.floor(v).astype(np.int64)
    fu, fv = u - i0, v - j0
    redge = r0 + dr * np.arange(nr + 1)
    area = 0.5 * dphi * (redge[1:] ** 2 - redge[:-1] ** 2)
    dfu = np.zeros(len(m))
    dfv = np.zeros(len(m))
    dm = np.zeros(len(m))
    for a in (0, 1):
        for b in (0, 1):
            i = i0 + a
            j = np.mod(j0 + b, nphi)
            ok = (i >= 0) & (i < nr)
            gb = np.zeros(len(m))
            gb[ok] = g[i[ok], j[ok]] / area[i[ok]]
            wu = fu if a else 1 - fu
            wv = fv if b else 1 - fv
            dm += gb * wu * wv
            dfu += gb * m * (1 if a else -1) * wv
            dfv += gb * m * wu * (1 if b else -1)
    du, dv = dfu / dr, dfv / dphi
    gpos = np.zeros_like(pos)
    gpos[idx, 0] = du * x / R - dv * y / R ** 2
    gpos[idx, 1] = du * y / R + dv * x / R ** 2
    gmass = np.zeros_like(m_all)
    gmass[idx] = dm
    return gpos, gmass


def kdk_positions(pos, vel, mass, dt, steps, force):
    """FP32 roundings of the positions at steps 0..K of leapfrog(): the
    inputs of the trees a tree-code run builds along its trajectory."""
    m = _f64(mass)
    x, v = _f64(pos).reshape(-1, 3), _f64(vel).reshape(-1, 3)
    out = [x.astype(np.float32)]
    for _ in range(steps):
        x, v = leapfrog(x, v, m, dt, 1, force)
        out.append(x.astype(np.float32))
    return out
