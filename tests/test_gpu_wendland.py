"""The Wendland C2 kernel (support 2h, h_fact 1.3: the kernel of the paper's
example applications, Sec. 3) through the same GPU path, against the FP64
oracle with the same kernel: density and h-rho solve, forces, adjoint.
Gates as for M4: 1e-5 (FP64 form) and 1e-3 (FP32 form) on rho, h, Omega and
on |a - a_oracle| / A_a, |du - du_oracle| / U_a; gradients 1e-6 / 1e-3 of
their largest entry."""
import os

import numpy as np
import pytest

import workloads as W
from _gpu import gpu_density, gpu_forces, oracle_density, oracle_forces, sample_balls
from test_gpu_adjoint import GTOL, _cluster, _cotangents, _gpu_grads, _oracle_grads, _rel

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-5, "fp32": 1e-3}
WC2 = dict(kernel=1, hfact=1.3)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "lattice_wc2.txt")


def _rmax(a, b):
    return float(np.max(np.abs(a - b) / np.abs(b)))


def _check_forces(gf, of, prec, idx=None):
    idx = slice(None) if idx is None else idx
    da = np.sqrt(sum((gf[k][idx] - of[k]) ** 2 for k in ("ax", "ay", "az")))
    assert np.max(da / of["anorm"]) < TOL[prec]
    assert np.max(np.abs(gf["dudt"][idx] - of["dudt"]) / np.maximum(of["unorm"], 1e-300)) < TOL[prec]
    assert np.max(np.abs(gf["vsig"][idx] - of["vsig"]) / of["vsig"]) < TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_lattice_closed_form(prec):
    # 16^3 lattice: 81 neighbours (self included) and the lattice h-rho
    # solution of the golden file, and the oracle's values per particle
    g0 = {l.split()[0]: float(l.split()[1]) for l in open(GOLDEN)
          if l.strip() and not l.startswith("#")}
    st, p = W.lattice_box()
    p = dict(p, **WC2)
    g, ctx, ds, (rho, om) = gpu_density(st, p, prec)
    o = oracle_density(st, p)
    assert g["failures"] == 0
    assert np.all(g["nneigh"] == int(g0["nneigh_incl_self"]))
    assert np.array_equal(g["nneigh"], o["nneigh"])
    for k in ("h", "rho", "omega"):
        assert _rmax(g[k], o[k]) < TOL[prec], k
    assert np.max(np.abs(g["h"] * 16 - g0["h_over_dx"])) < TOL[prec] * g0["h_over_dx"]
    assert np.max(np.abs(g["rho"] - g0["rho_over_rho0"])) < TOL[prec]
    gf = gpu_forces(ctx, ds, rho, om)
    of = oracle_forces(st, p, o["h"], o["rho"], o["omega"])
    _check_forces(gf, of, prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("nside", [23, 17])
def test_jittered_mixed_mass_box(prec, nside):
    # several tiles and a ragged tail; random velocities switch the viscosity on
    st, p = W.shock_box(nside=nside)
    p = dict(p, m0=1.0 / nside ** 3, **WC2)
    n = st["x"].shape[0]
    rng = np.random.default_rng(31)
    st = dict(st, vx=rng.normal(0, 0.3, n), vy=rng.normal(0, 0.3, n))
    g, ctx, ds, (rho, om) = gpu_density(st, p, prec)
    o = oracle_density(st, p)
    assert g["failures"] == 0 and o["failures"] == 0
    for k in ("h", "rho", "omega"):
        assert _rmax(g[k], o[k]) < TOL[prec], k
    gf = gpu_forces(ctx, ds, rho, om)
    of = oracle_forces(st, p, o["h"], o["rho"], o["omega"])
    _check_forces(gf, of, prec)


def test_small_disc_locally_isothermal():
    st, p = W.planet_disc(n=20000)
    p = dict(p, **WC2)
    g, ctx, ds, (rho, om) = gpu_density(st, p, "fp32")
    o = oracle_density(st, p)
    assert g["failures"] == 0 and o["failures"] == 0
    for k in ("h", "rho", "omega"):
        assert _rmax(g[k], o[k]) < TOL["fp32"], k
    gf = gpu_forces(ctx, ds, rho, om)
    of = oracle_forces(st, p, o["h"], o["rho"], o["omega"])
    _check_forces(gf, of, "fp32")


def test_full_size_box_sampled():
    # 64^3 = 262144 particles, FP32 form, the launch configuration of the
    # benchmark; the oracle solves the shells of 3 balls of 48 targets
    st, p = W.shock_box()
    p = dict(p, **WC2)
    n = st["x"].shape[0]
    rng = np.random.default_rng(4)
    st = dict(st, vx=rng.normal(0, 0.1, n), vz=rng.normal(0, 0.1, n))
    g, ctx, ds, (rho, om) = gpu_density(st, p, "fp32")
    assert g["failures"] == 0
    gf = gpu_forces(ctx, ds, rho, om)
    tg, shell = sample_balls(st, p, 3, 48, seed=5, hscale=1.3 / 64)
    o = oracle_density(st, p, targets=shell)
    ti = np.searchsorted(shell, tg)
    for k in ("h", "rho", "omega"):
        assert _rmax(g[k][tg], o[k][ti]) < TOL["fp32"], k
    h, r, w = np.full(n, 1e-9), np.ones(n), np.ones(n)
    h[shell], r[shell], w[shell] = o["h"], o["rho"], o["omega"]
    of = oracle_forces(st, p, h, r, w, targets=tg)
    _check_forces(gf, of, "fp32", idx=tg)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("eos", [2, 1])
def test_vjp_matches_oracle_gradient(prec, eos):
    st, p = _cluster(343, eos, 410 + eos, shift=1.3 if eos == 1 else 0.0)
    p = dict(p, **WC2)
    cot = _cotangents(st["x"].shape[0], 17)
    ox, om = _oracle_grads(st, p, cot)
    gx, gm = _gpu_grads(st, p, prec, cot)
    assert _rel(gx, ox) < GTOL[prec]
    assert _rel(gm, om) < GTOL[prec]
