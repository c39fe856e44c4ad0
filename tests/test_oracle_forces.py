"""Pins of the oracle's force, artificial viscosity and du/dt (no GPU).

Independent of the force formula itself:
 - with no viscosity and v = 0 the grad-h pressure force is minus the gradient
   of the thermal energy E = sum_b m_b u_b(rho_b) at fixed entropy, taken here
   by central differences of the converged density;
 - with no viscosity du_a/dt = (P_a / rho_a^2) d rho_a/dt, with d rho_a/dt a
   central difference of the converged density along the velocity field;
 - pairwise antisymmetry: total momentum and angular momentum are conserved
   and total energy is conserved with viscosity on;
 - on a perfect lattice the pressure force vanishes by symmetry;
 - the viscosity acts only on approaching pairs and only dissipates."""
import numpy as np
import pytest

import workloads as W

G = 5.0 / 3.0
# (kernel, h_fact): M4 at 1.2, Wendland C2 at 1.3 (the paper's pairings)
KERNELS = [pytest.param((0, 1.2), id="m4"), pytest.param((1, 1.3), id="wc2")]


def _cluster(orc, n=216, levels=(0, 1), vscale=0.0, seed_k=101, kern=(0, 1.2)):
    st, dx = W.random_cluster(n, seed_k=seed_k, levels=levels, vscale=vscale)
    d = orc.density(st["x"], st["y"], st["z"], st["level"], st["h"], m0=1.0, tol=1e-14,
                    max_iter=60, kernel=kern[0], hfact=kern[1])
    assert d["failures"] == 0
    return st, dx, d


def _forces(orc, st, d, u, kern=(0, 1.2), **kw):
    kw.setdefault("eos", 2)
    kw.setdefault("gamma", G)
    return orc.forces(st["x"], st["y"], st["z"], st["vx"], st["vy"], st["vz"], u, st["level"],
                      d["h"], d["rho"], d["omega"], m0=1.0, kernel=kern[0], **kw)


@pytest.mark.parametrize("kern", KERNELS)
def test_pressure_force_is_energy_gradient(orc, kern):
    st, dx, d = _cluster(orc, kern=kern)
    m = 2.0 ** -st["level"].astype(float)
    K = np.random.default_rng(7).uniform(1.0, 2.0, st["x"].shape[0])
    u = K * d["rho"] ** (G - 1) / (G - 1)
    f = _forces(orc, st, d, u, kern, alpha=0.0, beta=0.0)

    def energy(pos):
        dd = orc.density(pos[0], pos[1], pos[2], st["level"], d["h"], m0=1.0, tol=1e-14,
                         max_iter=60, kernel=kern[0], hfact=kern[1])
        assert dd["failures"] == 0
        return np.sum(m * K * dd["rho"] ** (G - 1) / (G - 1))

    pos = np.array([st["x"], st["y"], st["z"]])
    eps = 1e-6 * dx
    for a in (0, 37, 101, 150, 215):
        for k, key in enumerate(("ax", "ay", "az")):
            pp, pm = pos.copy(), pos.copy()
            pp[k, a] += eps
            pm[k, a] -= eps
            dEdx = (energy(pp) - energy(pm)) / (2 * eps)
            assert abs(m[a] * f[key][a] + dEdx) < 2e-6 * m[a] * f["anorm"][a]


@pytest.mark.parametrize("kern", KERNELS)
def test_dudt_is_pdv_work(orc, kern):
    st, dx, d = _cluster(orc, vscale=0.3, kern=kern)
    u = np.random.default_rng(8).uniform(1.0, 2.0, st["x"].shape[0])
    f = _forces(orc, st, d, u, kern, alpha=0.0, beta=0.0)
    pos = np.array([st["x"], st["y"], st["z"]])
    vel = np.array([st["vx"], st["vy"], st["vz"]])
    e = 1e-6
    kw = dict(m0=1.0, tol=1e-14, max_iter=60, kernel=kern[0], hfact=kern[1])
    rp = orc.density(*(pos + e * vel), st["level"], d["h"], **kw)
    rm = orc.density(*(pos - e * vel), st["level"], d["h"], **kw)
    drho = (rp["rho"] - rm["rho"]) / (2 * e)
    expect = (G - 1) * u / d["rho"] * drho
    assert np.max(np.abs(f["dudt"] - expect) / f["unorm"]) < 1e-6


@pytest.mark.parametrize("kern", KERNELS)
def test_conservation(orc, kern):
    st, dx, d = _cluster(orc, vscale=0.5, kern=kern)
    m = 2.0 ** -st["level"].astype(float)
    u = np.random.default_rng(9).uniform(1.0, 2.0, st["x"].shape[0])
    f = _forces(orc, st, d, u, kern, alpha=1.0, beta=2.0)
    a = np.array([f["ax"], f["ay"], f["az"]])
    x = np.array([st["x"], st["y"], st["z"]])
    v = np.array([st["vx"], st["vy"], st["vz"]])
    scale = np.sum(m * f["anorm"])
    assert np.max(np.abs((m * a).sum(axis=1))) < 1e-14 * scale
    L = np.cross(x.T, (m * a).T).sum(axis=0)
    assert np.max(np.abs(L)) < 1e-14 * np.sum(m * f["anorm"] * np.linalg.norm(x, axis=0))
    dE = np.sum(m * (np.sum(v * a, axis=0) + f["dudt"]))
    assert abs(dE) < 1e-14 * np.sum(m * (np.linalg.norm(v, axis=0) * f["anorm"] + f["unorm"]))


@pytest.mark.parametrize("kern", KERNELS)
def test_lattice_pressure_force_vanishes(orc, kern):
    st, p = W.lattice_box()
    d = orc.density(st["x"], st["y"], st["z"], st["level"], st["h"], m0=p["m0"], periodic=True,
                    lo=p["lo"], hi=p["hi"], tol=1e-13, kernel=kern[0], hfact=kern[1])
    z = np.zeros_like(st["x"])
    f = orc.forces(st["x"], st["y"], st["z"], z, z, z, None, st["level"], d["h"], d["rho"],
                   d["omega"], m0=p["m0"], eos=0, cs0=1.0, periodic=True, lo=p["lo"],
                   hi=p["hi"], kernel=kern[0])
    amax = np.max(np.abs([f["ax"], f["ay"], f["az"]]), axis=0)
    assert np.all(amax <= 1e-13 * f["anorm"])
    assert np.all(f["dudt"] == 0.0)


def test_viscosity_only_for_approaching_pairs(orc):
    st, dx, d = _cluster(orc)
    u = np.full(st["x"].shape[0], 1.5)
    c = np.array([st["x"].mean(), st["y"].mean(), st["z"].mean()])
    # expanding flow: every pair recedes, the viscosity must do nothing
    exp_ = dict(st, vx=0.3 * (st["x"] - c[0]), vy=0.3 * (st["y"] - c[1]),
                vz=0.3 * (st["z"] - c[2]))
    f_on = _forces(orc, exp_, d, u, alpha=1.0, beta=2.0)
    f_off = _forces(orc, exp_, d, u, alpha=0.0, beta=0.0)
    for k in ("ax", "ay", "az", "dudt"):
        assert np.array_equal(f_on[k], f_off[k])
    # contracting flow: the viscosity heats (sum m du/dt goes up) and brakes
    con = dict(st, vx=-exp_["vx"], vy=-exp_["vy"], vz=-exp_["vz"])
    f_on = _forces(orc, con, d, u, alpha=1.0, beta=2.0)
    f_off = _forces(orc, con, d, u, alpha=0.0, beta=0.0)
    m = 2.0 ** -st["level"].astype(float)
    assert np.sum(m * (f_on["dudt"] - f_off["dudt"])) > 0
    v = np.array([con["vx"], con["vy"], con["vz"]])
    da = np.array([f_on[k] - f_off[k] for k in ("ax", "ay", "az")])
    assert np.sum(m * np.sum(v * da, axis=0)) < 0


def test_eos_special_points(orc):
    x = np.array([1.0, 16.0, 3.0]); y = np.zeros(3)
    rho = np.array([2.0, 2.0, 0.5]); u = np.array([3.0, 3.0, 3.0])
    P, c = orc.eos(x, y, rho, u, eos=0, cs0=0.5)
    assert np.allclose(P, 0.25 * rho, rtol=0, atol=0) and np.all(c == 0.5)
    P, c = orc.eos(x, y, rho, u, eos=1, cs0=0.5, q_cs=0.25, r_ref=1.0)
    assert c[0] == 0.5 and c[1] == 0.25 and P[1] == 0.0625 * 2.0
    P, c = orc.eos(x, y, rho, u, eos=2, gamma=1.4)
    assert abs(P[2] - 0.4 * 0.5 * 3.0) < 1e-15 and abs(c[2] ** 2 - 1.4 * 0.4 * 3.0) < 1e-14
