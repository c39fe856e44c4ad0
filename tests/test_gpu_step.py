"""Whole leapfrog steps on the GPU vs the same kick-drift-kick sequence
composed from the oracle's functions, compared per particle id: the FP64
form over a few steps at 1e-9, and the FP32 form over the twenty steps of
the benchmarked box at a bound grown from its per-evaluation gate."""
import numpy as np
import pytest
import torch

import oracle
import paper_2409_11470_amd as A
import workloads as W
from _gpu import params_for

pytestmark = pytest.mark.gpu


def _orc_accel(st, p, sinks, G=1.0):
    d = oracle.density(st["x"], st["y"], st["z"], st["level"], st["h"], m0=p["m0"], tol=1e-12,
                       max_iter=60, periodic=p["periodic"], lo=p["lo"], hi=p["hi"])
    f = oracle.forces(st["x"], st["y"], st["z"], st["vx"], st["vy"], st["vz"], st["u"],
                      st["level"], d["h"], d["rho"], d["omega"], m0=p["m0"], eos=p["eos"],
                      cs0=p["cs0"], q_cs=p.get("q_cs", 0.25), r_ref=p.get("r_ref", 1.0),
                      gamma=p["gamma"], alpha=p["alpha"], beta=p["beta"],
                      periodic=p["periodic"], lo=p["lo"], hi=p["hi"])
    if sinks:
        oracle.sink_gravity(st["x"], st["y"], st["z"], [s["x"] for s in sinks],
                            [s["m"] for s in sinks], [s.get("eps", 0.0) for s in sinks], G,
                            f["ax"], f["ay"], f["az"])
    st["h"] = d["h"]
    return f


def _orc_steps(st, p, sinks, dt, nsteps):
    st = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()}
    f = _orc_accel(st, p, sinks)
    adiab = p["eos"] == 2
    for _ in range(nsteps):
        oracle.kick(st["vx"], st["vy"], st["vz"], st["u"] if adiab else None, f["ax"], f["ay"],
                    f["az"], f["dudt"] if adiab else None, 0.5 * dt)
        oracle.drift(st["x"], st["y"], st["z"], st["vx"], st["vy"], st["vz"], dt,
                     periodic=p["periodic"], lo=p["lo"], hi=p["hi"])
        f = _orc_accel(st, p, sinks)
        oracle.kick(st["vx"], st["vy"], st["vz"], st["u"] if adiab else None, f["ax"], f["ay"],
                    f["az"], f["dudt"] if adiab else None, 0.5 * dt)
    return st


def _gpu_steps(st, p, sinks, dt, nsteps, prec="fp64"):
    ctx = A.Context(params_for(p, prec))
    ds = A.DeviceState.from_numpy(st)
    A.apr_accel(ctx, ds, sinks)
    for k in range(nsteps):
        A.apr_step(ctx, ds, [], sinks, dt, k)
    A.apr_sync_status(ctx)
    g = ds.to_numpy()
    order = np.argsort(g["id"])
    return {k: (v[order] if isinstance(v, np.ndarray) else v) for k, v in g.items()}


def _check(g, o, keys=("x", "y", "z", "vx", "vy", "vz", "h", "u"), tol=1e-9):
    for k in keys:
        scale = max(np.max(np.abs(o[k])), 1e-30)
        err = np.max(np.abs(g[k] - o[k])) / scale
        assert err < tol, (k, err)


def test_box_steps():
    st, p = W.shock_box(nside=12)
    p = dict(p, m0=1.0 / 12 ** 3)
    dt = 0.3 * (1.2 / 12) / np.sqrt(5.0 / 3.0)
    g = _gpu_steps(st, p, [], dt, 3)
    o = _orc_steps(st, p, [], dt, 3)
    _check(g, o)


def test_disc_steps_with_sink():
    st, p = W.planet_disc(n=6000)
    g = _gpu_steps(st, p, p["sinks"], 2e-3, 3)
    o = _orc_steps(st, p, p["sinks"], 2e-3, 3)
    _check(g, o, keys=("x", "y", "z", "vx", "vy", "vz", "h"))


def test_steps_with_refinement_conserve_mass():
    # the disc's zone splits particles inside it during the step
    st, p = W.planet_disc(n=20000)
    ctx = A.Context(params_for(p, "fp64", r_sep_factor=0.5, nn_cap=0.0, split_mode=1, seed=3))
    ds = A.DeviceState.from_numpy(st)
    A.apr_accel(ctx, ds, p["sinks"])
    units = lambda lv: int(np.sum(2 ** (8 - lv.astype(np.int64))))
    m0 = units(ds.to_numpy()["level"])
    for k in range(3):
        A.apr_step(ctx, ds, p["zones"], p["sinks"], 2e-3, k)
    A.apr_sync_status(ctx)
    g = ds.to_numpy()
    assert units(g["level"]) == m0
    assert g["x"].shape[0] > st["x"].shape[0]
    # every particle inside the zone has reached its level
    c = np.array(p["zones"][0]["c"])
    r2 = (g["x"] - c[0]) ** 2 + (g["y"] - c[1]) ** 2 + (g["z"] - c[2]) ** 2
    assert np.all(g["level"][r2 < 0.9 ** 2] == 1)
    assert len(np.unique(g["id"])) == g["id"].shape[0]


def test_box_20_steps_fp32():
    # The benchmarked box's sequence (jittered lattice, left/right states,
    # adiabatic, AV), at 16^3 = 4096 particles, 20 KDK steps at the fixed
    # dt = 0.3 min(h / vsig) of t = 0, in the FP32 form against the FP64
    # oracle.  Each FP32 evaluation of a is accepted within eps = 1e-3 of the
    # L1 pair sum A (du/dt: of its sum U); with no growth beyond that, the
    # errors after n steps stay below
    #   v: n dt eps A_max,  x: n (n + 1)/2 dt^2 eps A_max,  u: n dt eps U_max,
    #   h: eps + 3 (x bound) / h_min  (h follows the positions);
    # the measured errors are far below these (FP32 evaluations agree to
    # about 1e-6), but a missing or doubled half kick, a wrong drift or a
    # wrong h carried between steps exceeds them.
    nside, n = 16, 20
    st, p = W.shock_box(nside=nside)
    p = dict(p, m0=1.0 / nside ** 3)
    f0 = _orc_accel({k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()},
                    p, [])
    vs = np.max(f0["vsig"])
    d0 = oracle.density(st["x"], st["y"], st["z"], st["level"], st["h"], m0=p["m0"], tol=1e-12,
                        max_iter=60, periodic=True, lo=p["lo"], hi=p["hi"])
    dt = 0.3 * np.min(d0["h"]) / vs
    g = _gpu_steps(st, p, [], dt, n, prec="fp32")
    o = _orc_steps(st, p, [], dt, n)
    # the L1 sums at the start and at the end (du/dt is zero at t = 0, v = 0,
    # and grows as the interface compresses)
    f1 = _orc_accel({k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in o.items()},
                    p, [])
    eps = 1e-3
    A_max = max(np.max(f0["anorm"]), np.max(f1["anorm"]))
    U_max = max(np.max(f0["unorm"]), np.max(f1["unorm"]))
    bound_v = n * dt * eps * A_max
    bound_x = 0.5 * n * (n + 1) * dt * dt * eps * A_max
    bound_u = n * dt * eps * U_max
    L = np.asarray(p["hi"], float) - np.asarray(p["lo"], float)
    dx = max(np.max(np.abs((g[k] - o[k]) - L[i] * np.round((g[k] - o[k]) / L[i])))
             for i, k in enumerate(("x", "y", "z")))
    dv = max(np.max(np.abs(g[k] - o[k])) for k in ("vx", "vy", "vz"))
    du = np.max(np.abs(g["u"] - o["u"]))
    dh = np.max(np.abs(g["h"] / o["h"] - 1))
    assert dx < bound_x and dv < bound_v and du < bound_u, (dx, bound_x, dv, bound_v, du,
                                                            bound_u)
    assert dh < eps + 3 * bound_x / np.min(o["h"]), dh
    # the steps did move the state: velocities grew from zero at the interface
    assert np.max(np.abs(o["vx"])) > 100 * bound_v / n
