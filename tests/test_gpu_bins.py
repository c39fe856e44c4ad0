"""Individual timesteps (paper Sec. 2.5) on the GPU (apr_bins_init,
apr_step_bins) against the oracle's step_bins: the FP64 form per id at 1e-9,
the FP32 form within bounds grown from its per-evaluation gate.

The 4000-particle planet disc with its sink and refinement zone, dt_max 0.5:
the Courant bins spread over 0..3 (8 substeps).  Two steps, compared per id
(children are numbered by their parents' ids on both sides): position,
velocity, u and h to 1e-9 of the largest value, level and bin exactly."""
import numpy as np
import pytest
import torch

import oracle
import paper_2409_11470_amd as A
import workloads as W
from _gpu import params_for

pytestmark = pytest.mark.gpu

DT, MAXB = 0.5, 6
SPLIT = dict(r_sep_factor=0.5, nn_cap=0.0, split_mode=1)


def _phys(p):
    return dict(m0=p["m0"], eos=p["eos"], cs0=p.get("cs0", 1.0), q_cs=p.get("q_cs", 0.25),
                r_ref=p.get("r_ref", 1.0), gamma=p.get("gamma", 5.0 / 3.0),
                alpha=p.get("alpha", 1.0), beta=p.get("beta", 2.0), hfact=p.get("hfact", 1.2),
                sinks=p.get("sinks", []), periodic=p["periodic"], lo=p["lo"], hi=p["hi"])


def _by_id(g):
    o = np.argsort(g["id"])
    return {k: (v[o] if isinstance(v, np.ndarray) else v) for k, v in g.items()}


def test_disc_steps_match_oracle():
    st, p = W.planet_disc(n=4000)
    n0 = st["x"].shape[0]
    phys = _phys(p)
    # oracle
    o = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()}
    oracle.accel_bins(o, **phys)
    o["bin"] = oracle.courant_bin(o["h"], o["vsig"], dt_max=DT, c_cfl=0.3, max_bin=MAXB)
    assert len(np.unique(o["bin"])) >= 3
    for step in range(2):
        o = oracle.step_bins(o, zones=p["zones"], dt_max=DT, step=step, max_bin=MAXB, seed=3,
                             **SPLIT, **phys)
    # GPU
    ctx = A.Context(params_for(p, "fp64", seed=3, **SPLIT))
    ds = A.DeviceState.from_numpy(st)
    A.apr_bins_init(ctx, ds, DT, 0.3, MAXB, p["sinks"])
    nsub = [A.apr_step_bins(ctx, ds, p["zones"], p["sinks"], DT, step, 0.3, MAXB)
            for step in range(2)]
    A.apr_sync_status(ctx)
    assert nsub[0] >= 4                  # bins 0..2 at least: 4 substeps or more
    g = _by_id(ds.to_numpy())
    o = _by_id(o)
    assert np.array_equal(g["id"], o["id"])
    assert int((g["id"] >= n0).sum()) > 10     # children were made
    for k in ("level", "bin"):
        assert np.array_equal(g[k], o[k]), k
    for k in ("x", "y", "z", "vx", "vy", "vz", "h", "u"):
        sc = max(np.max(np.abs(o[k])), 1e-30)
        assert np.max(np.abs(g[k] - o[k])) / sc < 1e-9, k


def _compare(g, o):
    g, o = _by_id(g), _by_id(o)
    assert np.array_equal(g["id"], o["id"])
    for k in ("level", "bin"):
        assert np.array_equal(g[k], o[k]), k
    L = np.asarray(o["hi"], float) - np.asarray(o["lo"], float) if "hi" in o else None
    for k in ("x", "y", "z", "vx", "vy", "vz", "h", "u"):
        d = g[k] - o[k]
        if L is not None and k in ("x", "y", "z"):
            w = L["xyz".index(k)]
            d -= w * np.round(d / w)          # periodic images
        sc = max(np.max(np.abs(o[k])), 1e-30)
        assert np.max(np.abs(d)) / sc < 1e-9, k


def test_wave_box_periodic_adiabatic():
    """The sound-wave box (periodic, adiabatic, cylinder zone), dt_max about
    twice the median Courant step: bins 1 and 2 (4 substeps), the u kicks and
    the periodic drift of the substeps, splits of active particles in the
    zone.  Two steps, per id against the oracle."""
    st, p = W.wave_box(nx=16)
    phys = _phys(p)
    o = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()}
    oracle.accel_bins(o, **phys)
    dtc = 0.3 * o["h"] / o["vsig"]
    dtm = 2.0 * float(np.median(dtc)) * 1.000123
    o["bin"] = oracle.courant_bin(o["h"], o["vsig"], dt_max=dtm, c_cfl=0.3, max_bin=MAXB)
    b0 = np.bincount(o["bin"])
    assert b0.size == 3 and b0[1] > 100 and b0[2] > 100
    for step in range(2):
        o = oracle.step_bins(o, zones=p["zones"], dt_max=dtm, step=step, max_bin=MAXB, seed=3,
                             **SPLIT, **phys)
    ctx = A.Context(params_for(p, "fp64", seed=3, **SPLIT))
    ds = A.DeviceState.from_numpy(st)
    A.apr_bins_init(ctx, ds, dtm, 0.3, MAXB)
    assert np.array_equal(np.bincount(ds["bin"].cpu().numpy()), b0)
    for step in range(2):
        k = int(ds["bin"].max())        # a step's end may refine past it
        assert A.apr_step_bins(ctx, ds, p["zones"], [], dtm, step, 0.3, MAXB) == 1 << k
        assert step > 0 or k == 2
    A.apr_sync_status(ctx)
    g = ds.to_numpy()
    assert int((g["id"] >= st["x"].shape[0]).sum()) > 10
    o["lo"], o["hi"] = p["lo"], p["hi"]
    _compare(g, o)


def test_periodic_drift_across_the_boundary():
    """The sound-wave box moving at 1.5 times its sound speed along x, no zone:
    nothing splits or merges, and during the substeps particles drift out of
    one side of the periodic box and in at the other.  Each substep sorts the
    cells again (a cell refitted to a wrapped particle would span the box):
    two steps per id against the oracle."""
    st, p = W.wave_box(nx=16, vx=1.5)
    phys = _phys(p)
    o = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()}
    oracle.accel_bins(o, **phys)
    dtc = 0.3 * o["h"] / o["vsig"]
    dtm = 2.0 * float(np.median(dtc)) * 1.000123
    o["bin"] = oracle.courant_bin(o["h"], o["vsig"], dt_max=dtm, c_cfl=0.3, max_bin=MAXB)
    assert np.bincount(o["bin"]).size >= 3          # bins 1 and 2 at least: 4 substeps
    for step in range(2):
        o = oracle.step_bins(o, zones=[], dt_max=dtm, step=step, max_bin=MAXB, seed=3,
                             **SPLIT, **phys)
    # particles that left through x = 1 and came back in at x = 0
    x0 = st["x"][np.argsort(st["id"])]
    xo = o["x"][np.argsort(o["id"])]
    assert int((xo < x0).sum()) > 50
    ctx = A.Context(params_for(p, "fp64", seed=3, **SPLIT))
    ds = A.DeviceState.from_numpy(st)
    A.apr_bins_init(ctx, ds, dtm, 0.3, MAXB)
    for step in range(2):
        assert A.apr_step_bins(ctx, ds, [], [], dtm, step, 0.3, MAXB) >= 4
    A.apr_sync_status(ctx)
    g = ds.to_numpy()
    assert g["x"].shape[0] == st["x"].shape[0]
    o["lo"], o["hi"] = p["lo"], p["hi"]
    _compare(g, o)


def test_argument_errors():
    st, p = W.planet_disc(n=2000)
    ctx = A.Context(params_for(p, "fp64", seed=3, **SPLIT))
    empty = A.DeviceState(8)
    bad = [lambda: A.apr_bins_init(ctx, empty, DT, 0.3, MAXB),
           lambda: A.apr_step_bins(ctx, empty, [], [], DT, 0, 0.3, MAXB)]
    ds = A.DeviceState.from_numpy(st)
    bad += [lambda: A.apr_bins_init(ctx, ds, 0.0, 0.3, MAXB),
            lambda: A.apr_bins_init(ctx, ds, DT, -1.0, MAXB),
            lambda: A.apr_bins_init(ctx, ds, DT, 0.3, 21)]
    for call in bad:
        with pytest.raises(A.AprError) as e:
            call()
        assert e.value.code == A.APR_ERR_INVALID
    A.apr_bins_init(ctx, ds, DT, 0.3, MAXB, p["sinks"])
    kmax = int(ds["bin"].max())
    assert kmax >= 2
    # a bin above the max_bin of the call, then a negative bin: rejected
    with pytest.raises(A.AprError) as e:
        A.apr_step_bins(ctx, ds, [], p["sinks"], DT, 0, 0.3, kmax - 1)
    assert e.value.code == A.APR_ERR_INVALID
    saved = ds["bin"][0].item()
    ds["bin"][0] = -1
    with pytest.raises(A.AprError) as e:
        A.apr_step_bins(ctx, ds, [], p["sinks"], DT, 0, 0.3, MAXB)
    assert e.value.code == A.APR_ERR_INVALID
    ds["bin"][0] = saved
    assert A.apr_step_bins(ctx, ds, [], p["sinks"], DT, 0, 0.3, MAXB) == 1 << kmax


def test_reorder_voids_the_stored_values():
    st, p = W.planet_disc(n=2000)
    ctx = A.Context(params_for(p, "fp64", seed=3, **SPLIT))
    ds = A.DeviceState.from_numpy(st)
    A.apr_bins_init(ctx, ds, DT, 0.3, MAXB, p["sinks"])
    A.apr_step_bins(ctx, ds, [], p["sinks"], DT, 0, 0.3, MAXB)
    A.apr_build_cells(ctx, ds)          # a reorder outside apr_step_bins
    with pytest.raises(A.AprError) as e:
        A.apr_step_bins(ctx, ds, [], p["sinks"], DT, 1, 0.3, MAXB)
    assert e.value.code == A.APR_ERR_INVALID
    A.apr_bins_init(ctx, ds, DT, 0.3, MAXB, p["sinks"])
    assert A.apr_step_bins(ctx, ds, [], p["sinks"], DT, 1, 0.3, MAXB) >= 1


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("fp32", 1e-4)])
def test_bin_zero_is_the_global_step(prec, tol):
    """With max_bin 0 every particle sits in bin 0: one substep, every
    particle active, i.e. apr_step's global step (random key step * 4096),
    per id to tol of the largest value, in both forms; in FP64 both also
    match the oracle.  The disc's velocity field has a divergence, so the h
    predicted for the next density pass differs from the last converged h
    that a split takes its offset and children's h from."""
    st, p = W.planet_disc(n=4000)
    out = []
    for bins in (True, False):
        ctx = A.Context(params_for(p, prec, seed=3, **SPLIT))
        ds = A.DeviceState.from_numpy(st, capacity=3 * st["x"].shape[0] + 64)
        if bins:
            A.apr_bins_init(ctx, ds, DT, 0.3, 0, p["sinks"])
            assert int(ds["bin"].max()) == 0
            for step in range(2):
                assert A.apr_step_bins(ctx, ds, p["zones"], p["sinks"], 0.05, step, 0.3, 0) == 1
        else:
            A.apr_accel(ctx, ds, p["sinks"])
            for step in range(2):
                A.apr_step(ctx, ds, p["zones"], p["sinks"], 0.05, step * 4096)
        A.apr_sync_status(ctx)
        out.append(_by_id(ds.to_numpy()))
    if prec == "fp64":
        # and both equal the oracle's global step (its bin-0 steps), whose
        # splits use the h of the last density pass
        phys = _phys(p)
        o = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()}
        oracle.accel_bins(o, **phys)
        o["bin"] = np.zeros(o["x"].shape[0], np.int8)
        for step in range(2):
            o = oracle.step_bins(o, zones=p["zones"], dt_max=0.05, step=step, max_bin=0,
                                 seed=3, **SPLIT, **phys)
        out.append(_by_id(o))
    for o in out[1:]:
        g = out[0]
        assert np.array_equal(g["id"], o["id"]) and np.array_equal(g["level"], o["level"])
        assert int((g["id"] >= st["x"].shape[0]).sum()) > 10
        for k in ("x", "y", "z", "vx", "vy", "vz", "h"):
            sc = max(np.max(np.abs(o[k])), 1e-30)
            assert np.max(np.abs(g[k] - o[k])) / sc < tol, k


def _l1_bounds(st, phys):
    """The largest L1 sums of the acceleration (hydro pair terms plus the sink
    pull) and of du/dt over the particles of a state, from the oracle."""
    box = dict(periodic=phys["periodic"], lo=phys["lo"], hi=phys["hi"])
    d = oracle.density(st["x"], st["y"], st["z"], st["level"], st["h"], m0=phys["m0"],
                       hfact=phys["hfact"], tol=1e-12, max_iter=60, **box)
    f = oracle.forces(st["x"], st["y"], st["z"], st["vx"], st["vy"], st["vz"], st.get("u"),
                      st["level"], d["h"], d["rho"], d["omega"], m0=phys["m0"], eos=phys["eos"],
                      cs0=phys["cs0"], q_cs=phys["q_cs"], r_ref=phys["r_ref"],
                      gamma=phys["gamma"], alpha=phys["alpha"], beta=phys["beta"], **box)
    a = f["anorm"]
    if phys["sinks"]:
        n = st["x"].shape[0]
        g = [np.zeros(n) for _ in range(3)]
        s = phys["sinks"]
        oracle.sink_gravity(st["x"], st["y"], st["z"], [q["x"] for q in s], [q["m"] for q in s],
                            [q.get("eps", 0.0) for q in s], 1.0, *g)
        a = a + np.sqrt(g[0] ** 2 + g[1] ** 2 + g[2] ** 2)
    return float(np.max(a)), float(np.max(f["unorm"])), float(np.min(d["h"]))


@pytest.mark.parametrize("case", ["wave", "disc"])
def test_fp32_steps_within_bounds(case):
    """The FP32 form of individual timesteps against the FP64 oracle: the wave
    box (periodic, adiabatic, cylinder zone, bins 1-2) and the planet disc
    (sink, sphere zone, bins 0-3), two steps of dt_max each.  Levels and bins
    exactly; the continuous values within bounds grown from the FP32 form's
    per-evaluation gate eps = 1e-3 of the L1 sums (A for the acceleration,
    hydro terms plus the sink pull; U for du/dt) over the time advanced,
    T = 2 dt_max:  v: T eps A_max,  x: T^2 eps A_max,  u: T eps U_max,
    h: eps + 3 (x bound) / h_min, with A_max, U_max the larger of the start's
    and the end's.  The measured errors are orders below (about 1e-7 of
    these scales); a missing or doubled kick, a substep drifted twice or a
    particle in the wrong bin exceeds them."""
    if case == "wave":
        st, p = W.wave_box(nx=16)
    else:
        st, p = W.planet_disc(n=4000)
    phys = _phys(p)
    o = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()}
    oracle.accel_bins(o, **phys)
    if case == "wave":
        dtm = 2.0 * float(np.median(0.3 * o["h"] / o["vsig"])) * 1.000123
    else:
        dtm = DT
    o["bin"] = oracle.courant_bin(o["h"], o["vsig"], dt_max=dtm, c_cfl=0.3, max_bin=MAXB)
    assert len(np.unique(o["bin"])) >= 2
    for step in range(2):
        o = oracle.step_bins(o, zones=p["zones"], dt_max=dtm, step=step, max_bin=MAXB, seed=3,
                             **SPLIT, **phys)
    ctx = A.Context(params_for(p, "fp32", seed=3, **SPLIT))
    ds = A.DeviceState.from_numpy(st)
    A.apr_bins_init(ctx, ds, dtm, 0.3, MAXB, p.get("sinks", []))
    for step in range(2):
        A.apr_step_bins(ctx, ds, p["zones"], p.get("sinks", []), dtm, step, 0.3, MAXB)
    A.apr_sync_status(ctx)
    g, o = _by_id(ds.to_numpy()), _by_id(o)
    assert np.array_equal(g["id"], o["id"])
    assert int((g["id"] >= st["x"].shape[0]).sum()) > 10     # children were made
    for k in ("level", "bin"):
        assert np.array_equal(g[k], o[k]), k
    a0, u0, h0 = _l1_bounds(st, phys)
    a1, u1, h1 = _l1_bounds(o, phys)
    eps, T = 1e-3, 2 * dtm
    A_max, U_max = max(a0, a1), max(u0, u1)
    bound = dict(x=T * T * eps * A_max, v=T * eps * A_max, u=T * eps * U_max)
    L = np.asarray(p["hi"], float) - np.asarray(p["lo"], float)
    for i, k in enumerate(("x", "y", "z")):
        d = g[k] - o[k]
        if p["periodic"]:
            d -= L[i] * np.round(d / L[i])
        assert np.max(np.abs(d)) < bound["x"], (k, np.max(np.abs(d)), bound["x"])
    for k in ("vx", "vy", "vz"):
        assert np.max(np.abs(g[k] - o[k])) < bound["v"], (k, bound["v"])
    if p["eos"] == 2:
        assert np.max(np.abs(g["u"] - o["u"])) < bound["u"], bound["u"]
    assert np.max(np.abs(g["h"] / o["h"] - 1)) < eps + 3 * bound["x"] / min(h0, h1)
