"""Pins of the oracle's velocity Verlet integrator (oracle/md.py) against
what the mathematics fixes: it is exact for a constant force, time
reversible, and its energy error for a harmonic potential is second order in
the step."""

import numpy as np

from oracle import md


def test_constant_force_exact():
    rng = np.random.default_rng(1)
    f = rng.normal(size=(3, 3))
    m = np.array([1.0, 2.5, 7.0])
    x0, v0 = rng.normal(size=(3, 3)), rng.normal(size=(3, 3))
    eg = lambda x: (float(-np.sum(f * x)), -f)
    dt, n = 0.37, 11
    x, v, ep, ek = md.velocity_verlet(eg, x0, v0, m, dt, n)
    t = dt * n
    a = f / m[:, None]
    assert np.max(np.abs(x - (x0 + v0 * t + 0.5 * a * t * t))) < 1e-12
    assert np.max(np.abs(v - (v0 + a * t))) < 1e-12
    assert np.max(np.abs((ep + ek) - (ep[0] + ek[0]))) < 1e-11     # exact for linear potentials


def _harmonic(k):
    return lambda x: (0.5 * float(np.sum(k * x * x)), k * x)


def test_harmonic_reversible():
    rng = np.random.default_rng(2)
    k = rng.uniform(0.5, 3.0, size=(4, 3))
    m = rng.uniform(1.0, 4.0, size=4)
    x0, v0 = rng.normal(size=(4, 3)), rng.normal(size=(4, 3))
    x, v, _, _ = md.velocity_verlet(_harmonic(k), x0, v0, m, 0.05, 200)
    xb, vb, _, _ = md.velocity_verlet(_harmonic(k), x, -v, m, 0.05, 200)
    assert np.max(np.abs(xb - x0)) < 1e-11 and np.max(np.abs(vb + v0)) < 1e-11


def test_harmonic_energy_error_second_order():
    k, m = np.array([[2.0, 2.0, 2.0]]), np.array([1.0])
    x0, v0 = np.array([[1.0, 0.0, -0.5]]), np.array([[0.0, 0.3, 0.0]])
    err = []
    for dt in (0.04, 0.02, 0.01):
        n = int(round(4.0 / dt))
        _, _, ep, ek = md.velocity_verlet(_harmonic(k), x0, v0, m, dt, n)
        e = ep + ek
        err.append(np.max(np.abs(e - e[0])))
    assert 3.5 < err[0] / err[1] < 4.5 and 3.5 < err[1] / err[2] < 4.5
