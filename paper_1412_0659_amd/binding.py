"""ctypes binding of the C ABI in include/bh.h.

Argument marshalling only: every step of the tree-code runs in the HIP
library libbh.so next to this file.  The entry points keep the C names
(bh_create, tree_build, tree_force, leapfrog_step, ...); torch supplies the
device memory (``tensor.data_ptr()``) and the stream
(``torch.cuda.current_stream().cuda_stream``).  There is no fallback: if the
library is missing, loading fails with an error that says how to build it.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libbh.so")

BH_OK, BH_EINVAL, BH_ECAPACITY, BH_ENOMEM, BH_EHIP, BH_ENONFINITE, BH_ESTATE, BH_EMASS = \
    0, -1, -2, -3, -4, -5, -6, -7

# export id -> (numpy dtype, values per element, element count kind)
EXPORTS = {
    "keys": (1, np.uint64, 1), "perm": (2, np.uint32, 1), "box": (3, np.float32, 1),
    "level_start": (4, np.uint32, 1), "cell_level": (5, np.uint32, 1),
    "cell_prefix": (6, np.uint64, 1), "cell_begin": (7, np.uint32, 1),
    "cell_count": (8, np.uint32, 1), "cell_child0": (9, np.uint32, 1),
    "cell_nchild": (10, np.uint32, 1), "cell_parent": (11, np.uint32, 1),
    "mom_M": (12, np.float64, 1), "mom_com": (13, np.float64, 3), "mom_Q": (14, np.float64, 6),
    "cell_comf": (15, np.float32, 4), "cell_size": (16, np.float32, 2),
    "group_begin": (17, np.uint32, 1), "group_count": (18, np.uint32, 1),
    "group_box": (19, np.float32, 8), "group_npp": (20, np.uint32, 1),
    "group_npc": (21, np.uint32, 1), "acc_sorted": (22, np.float32, 4),
    "boundary_flag": (23, np.uint32, 1), "boundary_cells": (24, np.uint32, 1),
    "boundary_box": (25, np.float32, 8), "let_origin": (26, np.uint32, 2),
    "let_node": (27, np.uint32, 2), "let_comf": (28, np.float32, 4),
}


class BhError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class bh_params(ctypes.Structure):
    _fields_ = [("nleaf", ctypes.c_int32), ("ncrit", ctypes.c_int32),
                ("far_fp16", ctypes.c_int32), ("pos_fp64", ctypes.c_int32),
                ("adjoint", ctypes.c_int32), ("curve", ctypes.c_int32),
                ("pair_groups", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class bh_cic_grid(ctypes.Structure):
    _fields_ = [("r_min", ctypes.c_float), ("r_max", ctypes.c_float),
                ("n_r", ctypes.c_int32), ("n_phi", ctypes.c_int32)]


class bh_stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("ncells", ctypes.c_int64), ("nleaves", ctypes.c_int64),
                ("ngroups", ctypes.c_int64), ("depth", ctypes.c_int64), ("n_pp", ctypes.c_int64),
                ("n_pc", ctypes.c_int64), ("ms_sort", ctypes.c_double),
                ("ms_build", ctypes.c_double), ("ms_moments", ctypes.c_double),
                ("ms_walk", ctypes.c_double), ("ms_step", ctypes.c_double),
                ("ms_walk_vjp", ctypes.c_double)]


class bh_tree_view(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("ncells", ctypes.c_int64), ("ngroups", ctypes.c_int64),
                ("level_start", ctypes.c_void_p), ("prefix", ctypes.c_void_p),
                ("level", ctypes.c_void_p), ("begin", ctypes.c_void_p), ("count", ctypes.c_void_p),
                ("child0", ctypes.c_void_p), ("nchild", ctypes.c_void_p),
                ("parent", ctypes.c_void_p), ("M", ctypes.c_void_p), ("S", ctypes.c_void_p),
                ("Q", ctypes.c_void_p), ("group_begin", ctypes.c_void_p)]


SYMBOLS = ["bh_create", "bh_destroy", "tree_build", "bh_set_state", "tree_force",
           "leapfrog_step", "bh_get_state", "bh_sync", "bh_stats_get", "bh_export",
           "bh_export_keys", "bh_export_tree",
           "bh_strerror", "bh_last_error", "tree_force_vjp", "leapfrog_vjp_drift",
           "bh_state_bytes", "bh_save_state", "bh_load_state", "bh_cic_density",
           "bh_cic_density_vjp", "tree_direct", "bh_diagnostics", "bh_set_box",
           "bh_decompose", "bh_decompose_sampled", "bh_domain_extract", "tree_force_add", "bh_boundary",
           "bh_let_build", "tree_force_let", "leapfrog_vjp_segment", "tree_force_static"]

_lib = None
_vp = ctypes.c_void_p


def load():
    """Load libbh.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                           "(run `python -c 'import __graft_entry__ as g; g.build()'`)")
    # torch's HIP runtime must be the one in the process before libbh.so binds
    # to libamdhip64.so.7: loading libbh.so first would bring in a second
    # runtime that torch then fails to initialise its devices with.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    i64, f32, c_int = ctypes.c_int64, ctypes.c_float, ctypes.c_int
    sig = {
        "bh_create": ([ctypes.POINTER(_vp), i64, ctypes.POINTER(bh_params)], c_int),
        "bh_destroy": ([_vp], c_int),
        "tree_build": ([_vp, _vp, _vp, i64, _vp], c_int),
        "bh_set_state": ([_vp, _vp, _vp, _vp, i64, _vp], c_int),
        "tree_force": ([_vp, f32, f32, _vp, _vp, _vp], c_int),
        "leapfrog_step": ([_vp, f32, f32, f32, _vp], c_int),
        "bh_get_state": ([_vp, _vp, _vp, _vp], c_int),
        "bh_sync": ([_vp, _vp], c_int),
        "bh_stats_get": ([_vp, ctypes.POINTER(bh_stats), _vp], c_int),
        "bh_export": ([_vp, c_int, _vp, i64, ctypes.POINTER(i64), _vp], c_int),
        "bh_export_keys": ([_vp, _vp, _vp, _vp], c_int),
        "bh_export_tree": ([_vp, ctypes.POINTER(bh_tree_view), _vp], c_int),
        "bh_strerror": ([c_int], ctypes.c_char_p),
        "bh_last_error": ([_vp], ctypes.c_char_p),
        "tree_force_vjp": ([_vp, f32, f32, _vp, f32, _vp, _vp, _vp], c_int),
        "leapfrog_vjp_drift": ([_vp, f32, _vp, _vp, _vp], c_int),
        "leapfrog_vjp_segment": ([_vp, _vp, i64, ctypes.c_int32, ctypes.c_int32, f32, f32, f32,
                                  _vp, _vp, _vp, _vp, _vp, _vp], c_int),
        "bh_state_bytes": ([_vp], i64),
        "bh_save_state": ([_vp, _vp, _vp], c_int),
        "bh_load_state": ([_vp, _vp, i64, _vp], c_int),
        "bh_cic_density": ([_vp, _vp, _vp, _vp, i64, ctypes.POINTER(bh_cic_grid), _vp, _vp],
                           c_int),
        "bh_cic_density_vjp": ([_vp, _vp, _vp, _vp, i64, ctypes.POINTER(bh_cic_grid), _vp, _vp,
                                _vp, _vp], c_int),
        "tree_direct": ([_vp, _vp, i64, f32, _vp, _vp, _vp], c_int),
        "bh_diagnostics": ([_vp, ctypes.POINTER(ctypes.c_double), _vp], c_int),
        "bh_set_box": ([_vp, _vp, f32], c_int),
        "bh_decompose": ([_vp, ctypes.c_int32, f32, _vp, _vp], c_int),
        "bh_decompose_sampled": ([_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_int32, f32, _vp, _vp, _vp], c_int),
        "bh_domain_extract": ([_vp, i64, i64, _vp, _vp, _vp, _vp, _vp], c_int),
        "tree_force_add": ([_vp, _vp, f32, f32, _vp, _vp, _vp], c_int),
        "bh_boundary": ([_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                         ctypes.POINTER(i64), _vp], c_int),
        "bh_let_build": ([_vp, _vp, ctypes.c_int32, f32, _vp, _vp], c_int),
        "tree_force_let": ([_vp, f32, f32, _vp, _vp, _vp, _vp], c_int),
        "tree_force_static": ([_vp, _vp, i64, f32, f32, _vp, _vp, _vp, _vp], c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _check(ctx, rc):
    if rc != BH_OK:
        L = load()
        msg = (L.bh_last_error(ctx) or b"").decode() if ctx else ""
        if not msg:
            msg = L.bh_strerror(rc).decode()
        raise BhError(rc, msg)


def _ptr(t):
    if t is None:
        return None
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous()
            and t.dtype == torch.float32):
        raise TypeError("expected a contiguous float32 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


# --- the C entry points, same names ------------------------------------------

CURVES = {"morton": 0, "ph": 1}


def bh_create(n_max: int, nleaf: int = 16, ncrit: int = 64, far_fp16: bool = False,
              pos_fp64: bool = False, adjoint: bool = False, curve: str = "morton",
              pair_groups: int = 0):
    p = bh_params(nleaf, ncrit, int(bool(far_fp16)), int(bool(pos_fp64)), int(bool(adjoint)),
                  CURVES[curve], int(pair_groups))
    out = _vp()
    rc = load().bh_create(ctypes.byref(out), int(n_max), ctypes.byref(p))
    _check(None, rc)
    return out


def bh_destroy(ctx):
    _check(None, load().bh_destroy(ctx))


def tree_build(ctx, pos, mass, stream=None):
    n = mass.shape[0]
    if pos.shape != (n, 3):
        raise ValueError("pos must be [N, 3]")
    _check(ctx, load().tree_build(ctx, _ptr(pos), _ptr(mass), n, _stream(stream)))


def bh_set_state(ctx, pos, vel, mass, stream=None):
    n = mass.shape[0]
    if pos.shape != (n, 3) or (vel is not None and vel.shape != (n, 3)):
        raise ValueError("pos and vel must be [N, 3]")
    _check(ctx, load().bh_set_state(ctx, _ptr(pos), _ptr(vel), _ptr(mass), n, _stream(stream)))


def tree_force(ctx, theta, eps, acc=None, pot=None, stream=None):
    _check(ctx, load().tree_force(ctx, float(theta), float(eps), _ptr(acc), _ptr(pot),
                                  _stream(stream)))


def leapfrog_step(ctx, dt, theta, eps, stream=None):
    _check(ctx, load().leapfrog_step(ctx, float(dt), float(theta), float(eps), _stream(stream)))


def bh_get_state(ctx, pos=None, vel=None, stream=None):
    _check(ctx, load().bh_get_state(ctx, _ptr(pos), _ptr(vel), _stream(stream)))


def bh_sync(ctx, stream=None):
    _check(ctx, load().bh_sync(ctx, _stream(stream)))


def bh_stats_get(ctx, stream=None) -> dict:
    st = bh_stats()
    _check(ctx, load().bh_stats_get(ctx, ctypes.byref(st), _stream(stream)))
    return {k: getattr(st, k) for k, _ in bh_stats._fields_}


def bh_export(ctx, name: str, count: int, stream=None) -> np.ndarray:
    aid, dt, width = EXPORTS[name]
    out = np.empty(count * width, dtype=dt)
    nb = ctypes.c_int64(0)
    _check(ctx, load().bh_export(ctx, aid, out.ctypes.data_as(_vp), out.nbytes, ctypes.byref(nb),
                                 _stream(stream)))
    k = nb.value // np.dtype(dt).itemsize
    out = out[:k]
    return out.reshape(-1, width) if width > 1 else out


def bh_export_keys(ctx, n: int, stream=None):
    """Sorted keys (u64) and permutation (u32) of the last build, host copies."""
    keys = np.empty(n, np.uint64)
    perm = np.empty(n, np.uint32)
    _check(ctx, load().bh_export_keys(ctx, keys.ctypes.data_as(_vp), perm.ctypes.data_as(_vp),
                                      _stream(stream)))
    return keys, perm


def bh_export_tree(ctx, stream=None) -> bh_tree_view:
    """Device views of the last built tree (pointers owned by the context)."""
    v = bh_tree_view()
    _check(ctx, load().bh_export_tree(ctx, ctypes.byref(v), _stream(stream)))
    return v


def _u8ptr(t):
    if t is None:
        return None
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous()
            and t.dtype in (torch.uint8, torch.bool)):
        raise TypeError("expected a contiguous uint8/bool CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


DIAG_FIELDS = ("mass", "kinetic", "potential", "px", "py", "pz", "lx", "ly", "lz")


def bh_diagnostics(ctx, stream=None) -> dict:
    """Total mass, kinetic and potential energy, momentum and angular
    momentum of the current state (FP64)."""
    out = (ctypes.c_double * len(DIAG_FIELDS))()
    _check(ctx, load().bh_diagnostics(ctx, out, _stream(stream)))
    return dict(zip(DIAG_FIELDS, list(out)))


def tree_direct(ctx, targets, eps, acc=None, pot=None, stream=None):
    """FP64 direct sum at caller indices `targets` (int64 CUDA tensor);
    returns (acc [nt,3], pot [nt]) as float64 CUDA tensors."""
    import torch
    if not (isinstance(targets, torch.Tensor) and targets.is_cuda and targets.is_contiguous()
            and targets.dtype == torch.int64):
        raise TypeError("expected a contiguous int64 CUDA tensor of targets")
    nt = targets.shape[0]
    if acc is None:
        acc = torch.empty((nt, 3), dtype=torch.float64, device=targets.device)
    if pot is None:
        pot = torch.empty((nt,), dtype=torch.float64, device=targets.device)
    for t in (acc, pot):
        if not (t.is_cuda and t.is_contiguous() and t.dtype == torch.float64):
            raise TypeError("expected contiguous float64 CUDA outputs")
    _check(ctx, load().tree_direct(ctx, ctypes.c_void_p(targets.data_ptr()), nt, float(eps),
                                   ctypes.c_void_p(acc.data_ptr()),
                                   ctypes.c_void_p(pot.data_ptr()), _stream(stream)))
    return acc, pot


def tree_force_vjp(ctx, theta, eps, u, coef, g_pos=None, g_mass=None, stream=None):
    _check(ctx, load().tree_force_vjp(ctx, float(theta), float(eps), _ptr(u), float(coef),
                                      _ptr(g_pos), _ptr(g_mass), _stream(stream)))


def leapfrog_vjp_drift(ctx, dt, gx, gv, stream=None):
    _check(ctx, load().leapfrog_vjp_drift(ctx, float(dt), _ptr(gx), _ptr(gv), _stream(stream)))


BH_SEG_FIRST, BH_SEG_LAST = 1, 2


def leapfrog_vjp_segment(ctx, snap, n, k, flags, dt, theta, eps, gx, gv, gx0=None, gv0=None,
                         gm=None, stream=None):
    """Reverse sweep of k leapfrog steps from the snapshot `snap` (uint8
    device tensor); gx0 / gv0 default to gx / gv (in place), gm accumulates."""
    import torch
    if not (isinstance(snap, torch.Tensor) and snap.is_cuda and snap.is_contiguous()):
        raise TypeError("expected a contiguous CUDA snapshot tensor")
    gx0 = gx if gx0 is None else gx0
    gv0 = gv if gv0 is None else gv0
    _check(ctx, load().leapfrog_vjp_segment(ctx, ctypes.c_void_p(snap.data_ptr()), int(n), int(k),
                                            int(flags), float(dt), float(theta), float(eps),
                                            _ptr(gx), _ptr(gv), _ptr(gx0), _ptr(gv0), _ptr(gm),
                                            _stream(stream)))


def bh_state_bytes(ctx) -> int:
    return int(load().bh_state_bytes(ctx))


def bh_save_state(ctx, dst, stream=None):
    import torch
    if not (isinstance(dst, torch.Tensor) and dst.is_cuda and dst.is_contiguous()
            and dst.dtype == torch.uint8 and dst.numel() >= bh_state_bytes(ctx)):
        raise TypeError("expected a large enough contiguous uint8 CUDA tensor")
    _check(ctx, load().bh_save_state(ctx, ctypes.c_void_p(dst.data_ptr()), _stream(stream)))


def bh_load_state(ctx, src, n, stream=None):
    _check(ctx, load().bh_load_state(ctx, ctypes.c_void_p(src.data_ptr()), int(n),
                                     _stream(stream)))


def bh_cic_density(ctx, pos, mass, sel, grid, density, stream=None):
    g = bh_cic_grid(*grid)
    _check(ctx, load().bh_cic_density(ctx, _ptr(pos), _ptr(mass), _u8ptr(sel), mass.shape[0],
                                      ctypes.byref(g), _ptr(density), _stream(stream)))


def bh_cic_density_vjp(ctx, pos, mass, sel, grid, g_density, g_pos=None, g_mass=None,
                       stream=None):
    g = bh_cic_grid(*grid)
    _check(ctx, load().bh_cic_density_vjp(ctx, _ptr(pos), _ptr(mass), _u8ptr(sel), mass.shape[0],
                                          ctypes.byref(g), _ptr(g_density), _ptr(g_pos),
                                          _ptr(g_mass), _stream(stream)))


def _u32ptr(t):
    if t is None:
        return None
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous()
            and t.dtype in (torch.int32, torch.uint32)):
        raise TypeError("expected a contiguous 32-bit integer CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def bh_set_box(ctx, lo=None, side=1.0):
    """Key later builds in the cube [lo, lo + side)^3 (lo None: own box)."""
    if lo is None:
        _check(ctx, load().bh_set_box(ctx, None, 1.0))
        return
    a = (ctypes.c_float * 3)(*[float(v) for v in np.asarray(lo, np.float32).reshape(3)])
    _check(ctx, load().bh_set_box(ctx, ctypes.cast(a, _vp), float(side)))


def bh_decompose(ctx, p, cap=1.3, stream=None) -> np.ndarray:
    """Cuts [p + 1] of the sorted particles into p flop-balanced domains."""
    cuts = np.zeros(int(p) + 1, np.int64)
    _check(ctx, load().bh_decompose(ctx, int(p), float(cap), cuts.ctypes.data_as(_vp),
                                    _stream(stream)))
    return cuts


def bh_decompose_sampled(ctx, px, py, m1, m2, cap=1.3, stream=None):
    """Cuts [p + 1] and boundary keys [p - 1] of the two-level sampling."""
    p = int(px) * int(py)
    cuts = np.zeros(p + 1, np.int64)
    bounds = np.zeros(max(p - 1, 1), np.uint64)
    _check(ctx, load().bh_decompose_sampled(ctx, int(px), int(py), int(m1), int(m2), float(cap),
                                            cuts.ctypes.data_as(_vp), bounds.ctypes.data_as(_vp),
                                            _stream(stream)))
    return cuts, bounds[:p - 1]


def bh_domain_extract(ctx, lo, hi, pos=None, vel=None, mass=None, ids=None, stream=None):
    _check(ctx, load().bh_domain_extract(ctx, int(lo), int(hi), _ptr(pos), _ptr(vel),
                                         _ptr(mass), _u32ptr(ids), _stream(stream)))


def tree_force_add(ctx, src, theta, eps, acc=None, pot=None, stream=None):
    _check(ctx, load().tree_force_add(ctx, src, float(theta), float(eps), _ptr(acc), _ptr(pot),
                                      _stream(stream)))


def bh_boundary(ctx, max_cells, stream=None):
    """Boundary tree; returns (level, number of terminal cells)."""
    lev = ctypes.c_int32(0)
    nt = ctypes.c_int64(0)
    _check(ctx, load().bh_boundary(ctx, int(max_cells), ctypes.byref(lev), ctypes.byref(nt),
                                   _stream(stream)))
    return lev.value, nt.value


def bh_let_build(ctx, srcs, theta, stream=None) -> np.ndarray:
    """Merged LETs of the source contexts; returns info [nsrc][3]:
    (boundary tree sufficed, LET cells, LET particles)."""
    k = len(srcs)
    arr = (_vp * max(k, 1))(*[s.value if isinstance(s, _vp) else s for s in srcs])
    info = np.zeros((max(k, 1), 3), np.int64)
    _check(ctx, load().bh_let_build(ctx, ctypes.cast(arr, _vp) if k else None, k, float(theta),
                                    info.ctypes.data_as(_vp), _stream(stream)))
    return info[:k]


def tree_force_let(ctx, theta, eps, rows=None, acc=None, pot=None, stream=None):
    _check(ctx, load().tree_force_let(ctx, float(theta), float(eps), _u32ptr(rows), _ptr(acc),
                                      _ptr(pot), _stream(stream)))


BH_STATIC_MAX_N = 65536


def tree_force_static(pos, mass, theta, eps, acc=None, pot=None, status=None, stream=None):
    """tree_build + tree_force without a context or any allocation (the
    library's static device buffer; n <= BH_STATIC_MAX_N).  status: an
    optional one-element int32 CUDA tensor receiving the device status bits."""
    n = mass.shape[0]
    if pos.shape != (n, 3):
        raise ValueError("pos must be [N, 3]")
    _check(None, load().tree_force_static(_ptr(pos), _ptr(mass), n, float(theta), float(eps),
                                          _ptr(acc), _ptr(pot), _u32ptr(status),
                                          _stream(stream)))


class Tree:
    """Owns one library context; methods call the C entry points."""

    def __init__(self, n_max: int, nleaf: int = 16, ncrit: int = 64, far_fp16: bool = False,
                 pos_fp64: bool = False, adjoint: bool = False, curve: str = "morton",
                 pair_groups: int = 0):
        self.ctx = bh_create(n_max, nleaf, ncrit, far_fp16, pos_fp64, adjoint, curve,
                             pair_groups)
        self.n = 0
        self.pos_fp64 = bool(pos_fp64)

    def save(self):
        """Exact snapshot of the state (device bytes)."""
        import torch
        buf = torch.empty(bh_state_bytes(self.ctx), dtype=torch.uint8, device="cuda")
        bh_save_state(self.ctx, buf)
        return buf

    def snapshot_bytes(self, n) -> int:
        """Size of a snapshot of n particles for this context's layout."""
        return int(n) * (32 + (24 if self.pos_fp64 else 0))

    def restore(self, buf, n=None):
        k = self.n if n is None else n
        if buf.numel() * buf.element_size() != self.snapshot_bytes(k):
            raise ValueError("snapshot size does not match this context and n")
        bh_load_state(self.ctx, buf, k)
        if n is not None:
            self.n = n

    def diagnostics(self) -> dict:
        return bh_diagnostics(self.ctx)

    def save_file(self, path):
        """Write an exact snapshot of the state (restart point) to `path` (.npz)."""
        import numpy as np
        buf = self.save()
        np.savez(path, state=buf.cpu().numpy(), n=np.int64(self.n))

    def load_file(self, path):
        """Restore a snapshot written by save_file (same n_max and parameters)."""
        import numpy as np
        import torch
        with np.load(path, allow_pickle=False) as z:
            n = int(z["n"])
            buf = torch.from_numpy(z["state"]).to("cuda")
        self.restore(buf, n)

    def direct(self, targets, eps):
        return tree_direct(self.ctx, targets, eps)

    def force_vjp(self, theta, eps, u, coef=1.0, g_pos=None, g_mass=None):
        tree_force_vjp(self.ctx, theta, eps, u, coef, g_pos, g_mass)

    def close(self):
        if self.ctx:
            bh_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def build(self, pos, mass):
        tree_build(self.ctx, pos, mass)
        self.n = mass.shape[0]

    def set_state(self, pos, vel, mass):
        bh_set_state(self.ctx, pos, vel, mass)
        self.n = mass.shape[0]

    def force(self, theta, eps, acc=None, pot=None):
        import torch
        if acc is None:
            acc = torch.empty((self.n, 3), dtype=torch.float32, device="cuda")
        if pot is None:
            pot = torch.empty((self.n,), dtype=torch.float32, device="cuda")
        tree_force(self.ctx, theta, eps, acc, pot)
        return acc, pot

    def step(self, dt, theta, eps):
        leapfrog_step(self.ctx, dt, theta, eps)

    def state(self):
        import torch
        pos = torch.empty((self.n, 3), dtype=torch.float32, device="cuda")
        vel = torch.empty((self.n, 3), dtype=torch.float32, device="cuda")
        bh_get_state(self.ctx, pos, vel)
        return pos, vel

    def sync(self):
        bh_sync(self.ctx)

    def stats(self) -> dict:
        return bh_stats_get(self.ctx)

    def export(self, name: str) -> np.ndarray:
        st = self.stats()
        sizes = {"keys": st["n"], "perm": st["n"], "acc_sorted": st["n"], "box": 5,
                 "level_start": 23}
        if name.startswith("cell") or name.startswith("mom") or name == "boundary_flag":
            count = st["ncells"]
        elif name.startswith("group"):
            count = st["ngroups"]
        elif name.startswith("boundary"):
            count = self.nterm
        elif name.startswith("let"):
            count = self.let_cells
        else:
            count = sizes[name]
        return bh_export(self.ctx, name, count)

    # ---- several domains on one device (Sec. III.B)

    def set_box(self, lo=None, side=1.0):
        bh_set_box(self.ctx, lo, side)

    def decompose(self, p, cap=1.3) -> np.ndarray:
        return bh_decompose(self.ctx, p, cap)

    def decompose_sampled(self, px, py, m1, m2, cap=1.3):
        return bh_decompose_sampled(self.ctx, px, py, m1, m2, cap)

    def extract(self, lo, hi):
        """Particles of sorted slots [lo, hi): (pos, vel, mass, ids) tensors."""
        import torch
        k = int(hi) - int(lo)
        pos = torch.empty((k, 3), dtype=torch.float32, device="cuda")
        vel = torch.empty((k, 3), dtype=torch.float32, device="cuda")
        mass = torch.empty((k,), dtype=torch.float32, device="cuda")
        ids = torch.empty((k,), dtype=torch.int32, device="cuda")
        bh_domain_extract(self.ctx, lo, hi, pos, vel, mass, ids)
        return pos, vel, mass, ids

    def force_add(self, src, theta, eps, acc, pot):
        tree_force_add(self.ctx, src.ctx, theta, eps, acc, pot)

    def boundary(self, max_cells):
        self.boundary_level, self.nterm = bh_boundary(self.ctx, max_cells)
        return self.boundary_level, self.nterm

    def let_build(self, srcs, theta) -> np.ndarray:
        info = bh_let_build(self.ctx, [s.ctx for s in srcs], theta)
        self.let_cells = int(self.let_virtual(len(srcs)) + info[:, 1].sum()) if srcs else 0
        return info

    @staticmethod
    def let_virtual(k) -> int:
        """Virtual cells above k LET roots (levels of at most 8 children)."""
        sizes = [k]
        while sizes[0] > 1 or len(sizes) == 1:
            sizes.insert(0, (sizes[0] + 7) // 8)
        return sum(sizes[:-1])

    def force_let(self, theta, eps, rows=None, acc=None, pot=None, stream=None):
        import torch
        if acc is None:
            acc = torch.empty((self.n, 3), dtype=torch.float32, device="cuda")
        if pot is None:
            pot = torch.empty((self.n,), dtype=torch.float32, device="cuda")
        tree_force_let(self.ctx, theta, eps, rows, acc, pot, stream)
        return acc, pot
