"""Pins of the oracle's second-order leapfrog (Sec. III.B.2): the phase error
of a circular softened two-body orbit and the energy error scale as dt^2,
and the kick-drift-kick scheme is time reversible."""
import numpy as np

from workloads import ics


def _circular_pair(m1=1.0, m2=0.5, d=1.0, eps=0.1):
    M = m1 + m2
    w = np.sqrt(M / (d * d + eps * eps) ** 1.5)
    x1, x2 = -m2 / M * d, m1 / M * d
    pos = np.array([[x1, 0, 0], [x2, 0, 0]])
    vel = np.array([[0, x1 * w, 0], [0, x2 * w, 0]])
    return pos, vel, np.array([m1, m2]), w


def _phase_error(oracle, dt, T):
    pos, vel, m, w = _circular_pair()
    steps = int(round(T / dt))
    f = oracle.direct_force_fn(m, 0.1)
    x, _ = oracle.leapfrog(pos, vel, m, dt, steps, f)
    rel = x[1] - x[0]
    ang = np.arctan2(rel[1], rel[0])
    want = np.angle(np.exp(1j * w * steps * dt))
    return abs(np.angle(np.exp(1j * (ang - want))))


def test_phase_error_second_order(oracle):
    T = 6.0
    e1 = _phase_error(oracle, 0.02, T)
    e2 = _phase_error(oracle, 0.01, T)
    assert 3.5 <= e1 / e2 <= 4.5, (e1, e2)


def _energy(oracle, x, v, m, eps):
    _, pot = oracle.direct(x, m, eps)
    return 0.5 * (m * (v ** 2).sum(1)).sum() + 0.5 * (m * pot).sum()


def test_energy_error_second_order(oracle):
    s = ics.plummer(512, 21)
    m = s.mass.astype(np.float64)
    eps = 0.05
    f = oracle.direct_force_fn(m, eps)
    E0 = _energy(oracle, s.pos.astype(np.float64), s.vel.astype(np.float64), m, eps)
    errs = []
    for dt in (0.02, 0.01):
        x, v = oracle.leapfrog(s.pos, s.vel, m, dt, int(round(1.0 / dt)), f)
        errs.append(abs(_energy(oracle, x, v, m, eps) / E0 - 1))
    assert 3.0 <= errs[0] / errs[1] <= 5.0, errs


def test_time_reversible(oracle):
    s = ics.plummer(256, 22)
    m = s.mass.astype(np.float64)
    f = oracle.direct_force_fn(m, 0.05)
    x0 = s.pos.astype(np.float64)
    x, v = oracle.leapfrog(x0, s.vel, m, 0.01, 100, f)
    xb, _ = oracle.leapfrog(x, -v, m, 0.01, 100, f)
    assert np.abs(xb - x0).max() <= 1e-10
