"""GPU force / artificial viscosity / du/dt vs the FP64 oracle, per particle:
|a_gpu - a_oracle| / A_a and |du_gpu - du_oracle| / U_a, where A_a and U_a are
the oracle's L1 sums of the pair terms (a ~ 0 on lattices makes plain
relative errors meaningless).  Gates 1e-5 (FP64 form), 1e-3 (FP32 form)."""
import numpy as np
import pytest

import workloads as W
from _gpu import gpu_density, gpu_forces, oracle_density, oracle_forces, sample_balls

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-5, "fp32": 1e-3}


def _check(gf, of, prec, idx=None):
    idx = slice(None) if idx is None else idx
    da = np.sqrt(sum((gf[k][idx] - of[k]) ** 2 for k in ("ax", "ay", "az")))
    ea = np.max(da / of["anorm"])
    eu = np.max(np.abs(gf["dudt"][idx] - of["dudt"]) / np.maximum(of["unorm"], 1e-300))
    ev = np.max(np.abs(gf["vsig"][idx] - of["vsig"]) / of["vsig"])
    assert ea < TOL[prec], ea
    assert eu < TOL[prec], eu
    assert ev < TOL[prec], ev


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_lattice_box(prec):
    st, p = W.lattice_box()
    g, ctx, ds, (rho, om) = gpu_density(st, p, prec)
    gf = gpu_forces(ctx, ds, rho, om)
    o = oracle_density(st, p)
    of = oracle_forces(st, p, o["h"], o["rho"], o["omega"])
    _check(gf, of, prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_shock_box_mixed_mass(prec):
    st, p = W.shock_box(nside=23)
    p = dict(p, m0=1.0 / 23 ** 3)
    rng = np.random.default_rng(3)
    st = dict(st, vx=rng.normal(0, 0.3, st["x"].shape[0]), vy=rng.normal(0, 0.3, st["x"].shape[0]))
    g, ctx, ds, (rho, om) = gpu_density(st, p, prec)
    gf = gpu_forces(ctx, ds, rho, om)
    o = oracle_density(st, p)
    of = oracle_forces(st, p, o["h"], o["rho"], o["omega"])
    _check(gf, of, prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_small_disc_locally_isothermal(prec):
    st, p = W.planet_disc(n=20000)
    g, ctx, ds, (rho, om) = gpu_density(st, p, prec)
    gf = gpu_forces(ctx, ds, rho, om)
    o = oracle_density(st, p)
    of = oracle_forces(st, p, o["h"], o["rho"], o["omega"])
    _check(gf, of, prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_full_size_box_sampled(prec):
    st, p = W.shock_box()
    rng = np.random.default_rng(4)
    n = st["x"].shape[0]
    st = dict(st, vx=rng.normal(0, 0.1, n), vz=rng.normal(0, 0.1, n))
    g, ctx, ds, (rho, om) = gpu_density(st, p, prec)
    gf = gpu_forces(ctx, ds, rho, om)
    tg, shell = sample_balls(st, p, 3, 48, seed=5, hscale=1.2 / 64)
    o = oracle_density(st, p, targets=shell)
    h, r, w = np.full(n, 1e-9), np.ones(n), np.ones(n)
    h[shell], r[shell], w[shell] = o["h"], o["rho"], o["omega"]
    of = oracle_forces(st, p, h, r, w, targets=tg)
    _check(gf, of, prec, idx=tg)
