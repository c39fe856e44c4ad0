"""Pins of the oracle's density and h-rho solve (no GPU)."""
import os

import numpy as np
import pytest

import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# (kernel, h_fact, golden file): M4 at 1.2, Wendland C2 at 1.3
KERNELS = [pytest.param((0, 1.2, "lattice_m4.txt"), id="m4"),
           pytest.param((1, 1.3, "lattice_wc2.txt"), id="wc2")]


def _golden(fname="lattice_m4.txt"):
    vals = {}
    for l in open(os.path.join(GOLDEN, fname)):
        if l.startswith("#") or not l.strip():
            continue
        k, v = l.split()
        vals[k] = float(v)
    return vals


def _dens(orc, st, p, **kw):
    return orc.density(st["x"], st["y"], st["z"], st["level"], st["h"], m0=p["m0"],
                       periodic=p["periodic"], lo=p["lo"], hi=p["hi"], **kw)


@pytest.mark.parametrize("kern", KERNELS)
def test_lattice_closed_form(orc, kern):
    g = _golden(kern[2])
    st, p = W.lattice_box()
    d = _dens(orc, st, p, tol=1e-13, kernel=kern[0], hfact=kern[1])
    dx = 1.0 / 16
    assert d["failures"] == 0
    assert np.all(d["nneigh"] == int(g["nneigh_incl_self"]))
    assert np.max(np.abs(d["h"] / dx - g["h_over_dx"])) < 1e-11
    assert np.max(np.abs(d["rho"] - g["rho_over_rho0"])) < 1e-11
    assert np.max(np.abs(d["omega"] - g["omega"])) < 1e-9
    # every particle of a lattice is alike; nearest neighbour at dx
    assert np.max(np.abs(d["dnn"] - dx)) < 1e-15
    # Newton from the guess 1.2 dx converges quadratically: M4 (3e-4 off)
    # needs 3 sums to reach 1e-13, Wendland C2 (7e-2 off) a few more
    assert d["iters"].max() <= (4 if kern[0] == 0 else 7)


@pytest.mark.parametrize("kern", KERNELS)
def test_lattice_fixed_h(orc, kern):
    # one Newton sum at h = h_fact dx exactly (max_iter = 1 reports the first sums)
    g = _golden(kern[2])
    st, p = W.lattice_box()
    st = dict(st, h=np.full_like(st["h"], kern[1] / 16))
    d = _dens(orc, st, p, max_iter=1, kernel=kern[0], hfact=kern[1])
    assert np.max(np.abs(d["rho"] - g["rho_over_rho0_at_h%g" % kern[1]])) < 1e-12


@pytest.mark.parametrize("kern", KERNELS)
def test_h_rho_relation_holds(orc, kern):
    st, p = W.shock_box(nside=12)
    p = dict(p, m0=1.0 / 12 ** 3)
    d = _dens(orc, st, p, tol=1e-13, kernel=kern[0], hfact=kern[1])
    m = p["m0"] / 2.0 ** st["level"]
    rel = np.abs(d["rho"] - m * (kern[1] / d["h"]) ** 3) / d["rho"]
    assert d["failures"] == 0 and rel.max() < 1e-11


def test_mass_scaling_and_translation(orc):
    # all masses halved -> rho halves at the same h; a periodic shift changes nothing
    st, p = W.shock_box(nside=10)
    p = dict(p, m0=1e-3)
    d0 = _dens(orc, st, p, tol=1e-13)
    st1 = dict(st, level=(st["level"] + 1).astype(np.int8))
    d1 = _dens(orc, st1, p, tol=1e-13)
    assert np.max(np.abs(d1["h"] / d0["h"] - 1)) < 1e-11
    assert np.max(np.abs(d1["rho"] / d0["rho"] - 0.5)) < 1e-11
    st2 = dict(st, x=np.mod(st["x"] + 0.37, 1.0), y=np.mod(st["y"] + 0.61, 1.0))
    d2 = _dens(orc, st2, p, tol=1e-13)
    assert np.max(np.abs(d2["rho"] / d0["rho"] - 1)) < 1e-10


def test_length_scaling(orc):
    # positions scaled by s (non-periodic) -> h scales by s, rho by s^-3
    st, dx = W.random_cluster(300, levels=(0, 1))
    p = dict(m0=1.0, periodic=False, lo=(0, 0, 0), hi=(1, 1, 1))
    d0 = _dens(orc, st, p, tol=1e-13)
    s = 2.5
    st1 = dict(st, x=st["x"] * s, y=st["y"] * s, z=st["z"] * s, h=st["h"] * s)
    d1 = _dens(orc, st1, p, tol=1e-13)
    assert np.max(np.abs(d1["h"] / (s * d0["h"]) - 1)) < 1e-10
    assert np.max(np.abs(d1["rho"] * s ** 3 / d0["rho"] - 1)) < 1e-10


@pytest.mark.parametrize("kern", KERNELS)
def test_omega_matches_difference(orc, kern):
    # Omega = 1 + h/(3 rho) d rho_sum/dh at fixed positions, by a central
    # difference of the density sum (max_iter = 1 evaluates the sum at h_in)
    st, p = W.shock_box(nside=10)
    p = dict(p, m0=1e-3)
    kw = dict(kernel=kern[0], hfact=kern[1])
    d = _dens(orc, st, p, tol=1e-13, **kw)
    e = 1e-7
    up = _dens(orc, dict(st, h=d["h"] * (1 + e)), p, max_iter=1, **kw)
    dn = _dens(orc, dict(st, h=d["h"] * (1 - e)), p, max_iter=1, **kw)
    drho = (up["rho"] - dn["rho"]) / (2 * e * d["h"])
    om = 1.0 + d["h"] * drho / (3.0 * d["rho"])
    assert np.max(np.abs(om - d["omega"])) < 1e-6


def test_isolated_particle_reports_failure(orc):
    # a lone particle has no h-rho solution: h grows until max_iter
    x = np.array([0.5]); lev = np.zeros(1, np.int8)
    d = orc.density(x, x, x, lev, np.array([0.1]), m0=1.0, max_iter=5)
    assert d["failures"] == 1 and d["nneigh"][0] == 1 and np.isinf(d["dnn"][0])


def test_targets_subset_matches_full(orc):
    st, p = W.shock_box(nside=10)
    p = dict(p, m0=1e-3)
    full = _dens(orc, st, p, tol=1e-12)
    tg = np.array([0, 17, 333, 999])
    sub = orc.density(st["x"], st["y"], st["z"], st["level"], st["h"][tg], m0=p["m0"],
                      periodic=True, lo=p["lo"], hi=p["hi"], tol=1e-12, targets=tg)
    assert np.array_equal(sub["rho"], full["rho"][tg])


def test_neighbour_lists_brute_force(orc):
    # hand-checkable: three particles on a line, supports 2h = 1.2, 1.0, 2.0;
    # r_01 = 1 sits exactly on particle 1's support edge (strict: excluded)
    x = np.array([0.0, 1.0, 2.5]); z0 = np.zeros(3)
    h = np.array([0.6, 0.5, 1.0])
    g = orc.neighbours(x, z0, z0, h)
    assert [list(a) for a in g] == [[1], [], [1]]
    s = orc.neighbours(x, z0, z0, h, symmetric=True)
    assert [list(a) for a in s] == [[1], [0, 2], [1]]
