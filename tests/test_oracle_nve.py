"""Pins of the oracle's velocity-Verlet integrator (the MD loop around the
force field, Background section: LAMMPS updates velocities and positions of
local atoms every time step; Evaluation section: dt = 0.5 fs water, 1.0 fs
copper).  A 3-D harmonic oscillator has the closed-form trajectory
x(t) = x0 cos(wt) + v0/w sin(wt); velocity Verlet is second order, so the
position error at fixed time scales as dt^2 and the energy error stays
bounded and O(dt^2)."""
import numpy as np

import oracle


def _run(dt, T=40.0):
    k = 0.7           # eV / A^2
    m = np.array([2.0, 5.0])
    x0 = np.array([[0.3, -0.2, 0.1], [0.0, 0.5, -0.4]])
    v0 = np.array([[0.01, 0.0, -0.02], [0.0, 0.015, 0.0]])

    def force(x):
        return 0.5 * k * float((x * x).sum()), -k * x

    n = int(round(T / dt))
    x, v, hist = oracle.nve(x0, v0, m, force, dt, n)
    w = np.sqrt(k * oracle.FTM2V / m)[:, None]
    t = n * dt
    xa = x0 * np.cos(w * t) + v0 / w * np.sin(w * t)
    etot = np.array([a + b for a, b in hist])
    return np.abs(x - xa).max(), np.abs(etot - etot[0]).max()


def test_harmonic_oscillator_second_order():
    e1, de1 = _run(0.2)
    e2, de2 = _run(0.1)
    assert e1 < 1e-2
    assert 3.0 < e1 / e2 < 5.0          # dt^2 convergence of the trajectory
    assert 3.0 < de1 / de2 < 5.0        # dt^2 energy error


def test_wrap_keeps_positions_in_box():
    m = np.array([1.0])
    x, v, _ = oracle.nve(np.array([[9.9, 0.05, 5.0]]), np.array([[0.5, -0.5, 0.0]]), m,
                         lambda x: (0.0, np.zeros_like(x)), 1.0, 3, wrap_box=np.array([10.0, 10.0, 10.0]))
    assert np.all((x >= 0) & (x < 10.0))
    assert np.allclose(x, [[1.4, 8.55, 5.0]])
