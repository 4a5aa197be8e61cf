"""Conserved quantities (bh_diagnostics) against the oracle on seeded
states, energy and momentum over the 1M workload's ten steps, and restart
from a snapshot file reproducing a run bit for bit."""
import numpy as np
import pytest

from gpu_util import gpu_tree, to_dev
from workloads import ics

pytestmark = pytest.mark.gpu


def test_diagnostics_match_oracle(oracle):
    s = ics.disk_halo(3000, 12000, 81)
    theta, eps = 0.5, 0.01
    t = gpu_tree(s.pos, s.mass, vel=s.vel)
    d0 = t.diagnostics()
    assert np.isnan(d0["potential"])
    t.force(theta, eps)
    d = t.diagnostics()
    m = s.mass.astype(np.float64)
    x = s.pos.astype(np.float64)
    v = s.vel.astype(np.float64)
    assert abs(d["mass"] - m.sum()) <= 1e-12 * m.sum()
    ke = 0.5 * (m * (v * v).sum(1)).sum()
    assert abs(d["kinetic"] - ke) <= 1e-12 * ke
    scale_p = (m * np.linalg.norm(v, axis=1)).sum()
    p = (m[:, None] * v).sum(0)
    assert np.allclose([d["px"], d["py"], d["pz"]], p, rtol=0, atol=1e-12 * scale_p)
    L = (m[:, None] * np.cross(x, v)).sum(0)
    scale_l = (m * np.linalg.norm(x, axis=1) * np.linalg.norm(v, axis=1)).sum()
    assert np.allclose([d["lx"], d["ly"], d["lz"]], L, rtol=0, atol=1e-12 * scale_l)
    ot = oracle.build_tree(s.pos, s.mass)
    _, opot, _, _ = oracle.walk(ot, theta, eps)
    pe = 0.5 * (m * opot).sum()
    print(f"PE gpu {d['potential']:.9e} oracle {pe:.9e}", flush=True)
    assert abs(d["potential"] - pe) <= 1e-5 * abs(pe)
    assert t.diagnostics() == d   # fixed summation order
    t.close()


def test_full_size_ten_steps_conserve():
    """The 1M disk + halo workload, ten steps: energy and momentum drift."""
    import paper_1412_0659_amd as bh
    w = ics.WORKLOADS["disk_halo_1m"]
    s = ics.make("disk_halo_1m")
    t = bh.Tree(s.n)
    t.set_state(to_dev(s.pos), to_dev(s.vel), to_dev(s.mass))
    t.force(w["theta"], w["eps"])
    d0 = t.diagnostics()
    e0 = d0["kinetic"] + d0["potential"]
    for _ in range(w["steps"]):
        t.step(w["dt"], w["theta"], w["eps"])
    d1 = t.diagnostics()
    e1 = d1["kinetic"] + d1["potential"]
    m = s.mass.astype(np.float64)
    scale_p = (m * np.linalg.norm(s.vel.astype(np.float64), axis=1)).sum()
    dp = np.linalg.norm([d1["px"] - d0["px"], d1["py"] - d0["py"], d1["pz"] - d0["pz"]])
    print(f"10 steps: dE/E {abs(e1 / e0 - 1):.2e}, |dp|/sum m|v| {dp / scale_p:.2e}", flush=True)
    assert abs(e1 / e0 - 1) <= 1e-4
    assert dp <= 1e-4 * scale_p
    t.close()


@pytest.mark.parametrize("pos_fp64", [False, True])
def test_restart_from_file_is_bit_identical(tmp_path, pos_fp64):
    import paper_1412_0659_amd as bh
    s = ics.disk_halo(4000, 16000, 82)
    theta, eps, dt = 0.4, 0.005, 1e-3
    a = bh.Tree(s.n, pos_fp64=pos_fp64)
    a.set_state(to_dev(s.pos), to_dev(s.vel), to_dev(s.mass))
    for k in range(6):
        a.step(dt, theta, eps)
        if k == 2:
            a.save_file(tmp_path / "snap.npz")
    pa, va = (x.cpu().numpy() for x in a.state())
    b = bh.Tree(s.n, pos_fp64=pos_fp64)
    b.load_file(tmp_path / "snap.npz")
    for _ in range(3):
        b.step(dt, theta, eps)
    pb, vb = (x.cpu().numpy() for x in b.state())
    assert np.array_equal(pa, pb) and np.array_equal(va, vb)
    other = bh.Tree(s.n, pos_fp64=not pos_fp64)
    with pytest.raises(ValueError):
        other.load_file(tmp_path / "snap.npz")
    a.close(); b.close(); other.close()
