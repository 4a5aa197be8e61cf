"""Seeded synthetic initial conditions for the gravitational tree-code workloads.

This module only draws inputs: particle positions, velocities and masses.  It
holds none of the tree-code's arithmetic, so both the CPU oracle's tests and
the GPU path's tests/bench may use it.

Models (all in units with G = 1):

* ``plummer``: a Plummer sphere of total mass 1 and scale radius 1, equal
  masses, isotropic velocities drawn from the Plummer distribution function
  (radius by inverse CDF, speed by von Neumann rejection on q = v / v_esc with
  density q^2 (1 - q^2)^(7/2)).  The centre of mass and mean velocity are
  removed.
* ``disk_halo``: the stand-in for the paper's Milky Way model (Section IV:
  an exponential disk inside a dark-matter halo, with several times more halo
  than disk particles).  An exponential disk (surface density ~ exp(-R/h),
  vertical profile sech^2(z/z0)) of mass 0.1 plus a Hernquist halo of mass 1
  and scale radius 5, truncated at 20 scale radii.  Disk particles get the
  circular speed of the spherically enclosed mass plus 10% Gaussian
  dispersion; halo particles get isotropic Gaussian velocities whose
  dispersion comes from the spherical Jeans equation, capped at 0.95 of the
  local escape speed.

All sampling is FP64 with ``numpy.random.Generator(PCG64)``; components use
independent streams from ``SeedSequence(seed).spawn``; results are rounded to
FP32 (the precision the tree-code consumes).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Snapshot:
    pos: np.ndarray      # float32 [N, 3]
    vel: np.ndarray      # float32 [N, 3]
    mass: np.ndarray     # float32 [N]
    is_disk: np.ndarray  # bool [N] (False for single-component models)

    @property
    def n(self) -> int:
        return int(self.mass.shape[0])


def _rngs(seed: int, k: int):
    return [np.random.Generator(np.random.PCG64(s)) for s in np.random.SeedSequence(seed).spawn(k)]


def _isotropic(rng, n):
    z = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([s * np.cos(ph), s * np.sin(ph), z], axis=1)


def _finish(pos, vel, mass, is_disk) -> Snapshot:
    mtot = mass.sum()
    pos = pos - (mass[:, None] * pos).sum(0) / mtot
    vel = vel - (mass[:, None] * vel).sum(0) / mtot
    return Snapshot(pos.astype(np.float32), vel.astype(np.float32),
                    mass.astype(np.float32), is_disk)


def plummer(n: int, seed: int = 1) -> Snapshot:
    """Plummer sphere, M = 1, a = 1, m = 1/n (exact in FP32 for n a power of two)."""
    r_rng, d_rng, q_rng, v_rng = _rngs(seed, 4)
    x = 1.0 - r_rng.uniform(0.0, 1.0, n)          # (0, 1]
    r = 1.0 / np.sqrt(np.maximum(x ** (-2.0 / 3.0) - 1.0, 1e-300))
    pos = r[:, None] * _isotropic(d_rng, n)
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        qq = q_rng.uniform(0.0, 1.0, todo.size)
        yy = q_rng.uniform(0.0, 0.1, todo.size)
        ok = yy < qq * qq * (1.0 - qq * qq) ** 3.5
        q[todo[ok]] = qq[ok]
        todo = todo[~ok]
    speed = q * np.sqrt(2.0) * (1.0 + r * r) ** (-0.25)
    vel = speed[:, None] * _isotropic(v_rng, n)
    mass = np.full(n, 1.0 / n)
    return _finish(pos, vel, mass, np.zeros(n, dtype=bool))


# --- disk + halo -----------------------------------------------------------

DISK_MASS = 0.1
DISK_H = 1.0
DISK_Z0 = 0.1
DISK_RMAX = 10.0
DISK_ZMAX = 1.0
HALO_MASS = 1.0
HALO_A = 5.0
HALO_RMAX = 20.0 * HALO_A


def _hernquist_cum(r):
    return r * r / (r + HALO_A) ** 2


def _sample_disk(rng, n):
    R = rng.gamma(2.0, DISK_H, n)
    bad = R > DISK_RMAX
    while bad.any():
        R[bad] = rng.gamma(2.0, DISK_H, int(bad.sum()))
        bad = R > DISK_RMAX
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    z = DISK_Z0 * np.arctanh(2.0 * rng.uniform(0.0, 1.0, n) - 1.0)
    bad = ~(np.abs(z) <= DISK_ZMAX)
    while bad.any():
        z[bad] = DISK_Z0 * np.arctanh(2.0 * rng.uniform(0.0, 1.0, int(bad.sum())) - 1.0)
        bad = ~(np.abs(z) <= DISK_ZMAX)
    return R, ph, z


def _sample_halo(rng_r, rng_d, n):
    u = rng_r.uniform(0.0, _hernquist_cum(HALO_RMAX), n)
    su = np.sqrt(u)
    r = HALO_A * su / (1.0 - su)
    return r[:, None] * _isotropic(rng_d, n), r


def disk_halo(n_disk: int, n_halo: int, seed: int = 2) -> Snapshot:
    """Exponential disk (mass 0.1) + truncated Hernquist halo (mass 1, a = 5)."""
    rd, rhr, rhd, vd, vh = _rngs(seed, 5)
    R, ph, z = _sample_disk(rd, n_disk)
    cph, sph = np.cos(ph), np.sin(ph)
    dpos = np.stack([R * cph, R * sph, z], axis=1)
    hpos, hr = _sample_halo(rhr, rhd, n_halo)
    md = np.full(n_disk, DISK_MASS / max(n_disk, 1))
    mh = np.full(n_halo, HALO_MASS / max(n_halo, 1))

    # spherically enclosed mass of all particles, used for circular speeds
    rall = np.concatenate([np.sqrt((dpos ** 2).sum(1)), hr])
    mall = np.concatenate([md, mh])
    order = np.argsort(rall, kind="stable")
    rs = rall[order]
    cm = np.cumsum(mall[order])

    def menc(r):
        k = np.searchsorted(rs, r, side="right")
        return np.where(k > 0, cm[np.maximum(k - 1, 0)], 0.0)

    # disk: circular speed + 10% Gaussian dispersion in (R, phi, z)
    vc = np.sqrt(menc(R) / np.maximum(R, 1e-12))
    sig = 0.1 * vc
    vR = vd.normal(0.0, 1.0, n_disk) * sig
    vphi = vc + vd.normal(0.0, 1.0, n_disk) * sig
    vz = vd.normal(0.0, 1.0, n_disk) * sig
    dvel = np.stack([vR * cph - vphi * sph, vR * sph + vphi * cph, vz], axis=1)

    # halo: isotropic Jeans dispersion on a log grid, total enclosed mass from
    # the particles; escape speed from the same spherical mass profile.
    grid = np.geomspace(1e-3, HALO_RMAX, 4096)
    rho = 1.0 / (grid * (grid + HALO_A) ** 3)               # shape only
    mg = menc(grid)
    integrand = rho * mg / grid ** 2
    seg = 0.5 * (integrand[1:] + integrand[:-1]) * np.diff(grid)
    tail = np.concatenate([np.cumsum(seg[::-1])[::-1], [0.0]])
    sig2 = tail / rho
    dm = np.diff(np.concatenate([[0.0], mg]))
    outer = np.concatenate([np.cumsum((dm / grid)[::-1])[::-1][1:], [0.0]])
    pot = -(mg / grid + outer)
    s_h = np.sqrt(np.interp(hr, grid, sig2))
    vesc = np.sqrt(2.0 * np.abs(np.interp(hr, grid, pot)))
    hvel = vh.normal(0.0, 1.0, (n_halo, 3)) * s_h[:, None]
    sp = np.sqrt((hvel ** 2).sum(1))
    cap = 0.95 * vesc
    fac = np.where(sp > cap, cap / np.maximum(sp, 1e-300), 1.0)
    hvel = hvel * fac[:, None]

    pos = np.concatenate([dpos, hpos])
    vel = np.concatenate([dvel, hvel])
    mass = np.concatenate([md, mh])
    is_disk = np.concatenate([np.ones(n_disk, bool), np.zeros(n_halo, bool)])
    return _finish(pos, vel, mass, is_disk)


def subsample(n: int, k: int, seed: int) -> np.ndarray:
    """Seeded uniform subsample of k distinct indices out of n, sorted."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.choice(n, size=min(k, n), replace=False))


# Named workloads: (description, generator kwargs, eps, theta)
WORKLOADS = {
    "plummer_16k": dict(model="plummer", n=16384, seed=1, eps=0.01, theta=0.5),
    "disk_halo_1m": dict(model="disk_halo", n_disk=200_000, n_halo=800_000, seed=2,
                         eps=0.005, theta=0.4, dt=1e-3, steps=10),
    "disk_halo_13m": dict(model="disk_halo", n_disk=2_166_667, n_halo=10_833_333, seed=3,
                          eps=0.002, theta=0.4, dt=1e-3, steps=10),
    "disk_halo_4m": dict(model="disk_halo", n_disk=800_000, n_halo=3_200_000, seed=4,
                         eps=0.005, theta=0.4),
}


def make(name: str) -> Snapshot:
    w = WORKLOADS[name]
    if w["model"] == "plummer":
        return plummer(w["n"], w["seed"])
    return disk_halo(w["n_disk"], w["n_halo"], w["seed"])


def disk_halo_scaled(n: int, seed: int, disk_fraction: float = 0.2) -> Snapshot:
    """The disk + halo model at an arbitrary particle count (1:4 disk:halo)."""
    nd = int(round(n * disk_fraction))
    return disk_halo(nd, n - nd, seed)


def perturbed(s: Snapshot, seed: int, sigma: float = 0.02) -> Snapshot:
    """The same particles with seeded Gaussian offsets N(0, sigma^2) added to
    every disk position component: initial conditions for a target
    snapshot."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = s.pos.astype(np.float64)
    d = np.nonzero(s.is_disk)[0]
    pos[d] += sigma * rng.standard_normal((len(d), 3))
    return Snapshot(pos.astype(np.float32), s.vel.copy(), s.mass.copy(), s.is_disk.copy())


# The differentiation workload: disk + halo, 64 KDK steps, the squared error
# of the disk's face-on (R, phi) surface density against the density reached
# from perturbed initial conditions.
DIFF_WORKLOADS = {
    "disk_halo_1m_adjoint": dict(n=1_000_000, seed=5, target_seed=1005, eps=0.005, theta=0.4,
                                 dt=1e-3, steps=64, every=8, grid=(0.2, 4.0, 16, 32)),
    "disk_halo_4096_adjoint": dict(n=4096, seed=5, target_seed=1005, eps=0.005, theta=0.4,
                                   dt=1e-3, steps=64, every=8, grid=(0.2, 4.0, 8, 8)),
}
