"""Pins of the oracle's leapfrog and sink gravity (no GPU)."""
import numpy as np


def _kdk(orc, x, v, dt, nsteps, G=1.0):
    X = [x[0].copy(), x[1].copy(), x[2].copy()]
    V = [v[0].copy(), v[1].copy(), v[2].copy()]
    n = X[0].shape[0]

    def acc():
        a = [np.zeros(n), np.zeros(n), np.zeros(n)]
        orc.sink_gravity(X[0], X[1], X[2], [[0.0, 0.0, 0.0]], [1.0], [0.0], G, *a)
        return a

    a = acc()
    for _ in range(nsteps):
        orc.kick(V[0], V[1], V[2], None, *a, None, 0.5 * dt)
        orc.drift(X[0], X[1], X[2], V[0], V[1], V[2], dt)
        a = acc()
        orc.kick(V[0], V[1], V[2], None, *a, None, 0.5 * dt)
    return X, V


def test_circular_orbit(orc):
    # unit mass, circular orbit at R: |a| = 1/R^2, period 2 pi R^1.5
    R = np.array([1.0, 4.0])
    x = [R.copy(), np.zeros(2), np.zeros(2)]
    v = [np.zeros(2), np.sqrt(1.0 / R), np.zeros(2)]
    a = [np.zeros(2), np.zeros(2), np.zeros(2)]
    orc.sink_gravity(*x, [[0, 0, 0]], [1.0], [0.0], 1.0, *a)
    assert np.allclose(a[0], -1.0 / R ** 2, rtol=1e-15)
    nsteps = 2000
    dt = 2 * np.pi / nsteps
    X, V = _kdk(orc, x, v, dt, nsteps)
    r = np.sqrt(X[0] ** 2 + X[1] ** 2)
    E0 = 0.5 / R - 1.0 / R
    E = 0.5 * (V[0] ** 2 + V[1] ** 2) - 1.0 / r
    assert abs(E[0] / E0[0] - 1) < 1e-5          # second order: (dt)^2 energy error
    assert abs(X[0][0] - 1.0) < 1e-4 and abs(X[1][0]) < 1e-3   # one full orbit


def test_time_reversible(orc):
    x = [np.array([1.3]), np.array([0.2]), np.array([-0.1])]
    v = [np.array([0.1]), np.array([0.8]), np.array([0.05])]
    X, V = _kdk(orc, x, v, 0.01, 300)
    X2, V2 = _kdk(orc, X, [-V[0], -V[1], -V[2]], 0.01, 300)
    for k in range(3):
        assert abs(X2[k][0] - x[k][0]) < 1e-12


def test_periodic_drift_wraps(orc):
    x = np.array([0.99]); y = np.array([0.01]); z = np.array([0.5])
    orc.drift(x, y, z, np.array([0.02]), np.array([-0.02]), np.array([0.0]), 1.0,
              periodic=True)
    assert abs(x[0] - 0.01) < 1e-15 and abs(y[0] - 0.99) < 1e-15 and z[0] == 0.5
