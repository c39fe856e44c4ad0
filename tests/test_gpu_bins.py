"""Individual timesteps (paper Sec. 2.5) on the GPU (apr_bins_init,
apr_step_bins) against the oracle's step_bins, FP64 form.

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
    return dict(m0=p["m0"], eos=p["eos"], cs0=p["cs0"], q_cs=p.get("q_cs", 0.25),
                r_ref=p.get("r_ref", 1.0), gamma=p["gamma"], alpha=p["alpha"], beta=p["beta"],
                hfact=p["hfact"], sinks=p["sinks"], periodic=p["periodic"], lo=p["lo"],
                hi=p["hi"])


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


def test_reorder_voids_the_stored_values():
    st, p = W.planet_disc(n=2000)
    ctx = A.Context(params_for(p, "fp64", seed=3, **SPLIT))
    ds = A.DeviceState.from_numpy(st)
    A.apr_bins_init(ctx, ds, DT, 0.3, MAXB, p["sinks"])
    A.apr_step_bins(ctx, ds, [], p["sinks"], DT, 0, 0.3, MAXB)
    A.apr_build_cells(ctx, ds)          # a reorder outside the driver
    with pytest.raises(A.AprError) as e:
        A.apr_step_bins(ctx, ds, [], p["sinks"], DT, 1, 0.3, MAXB)
    assert e.value.code == A.APR_ERR_INVALID
    A.apr_bins_init(ctx, ds, DT, 0.3, MAXB, p["sinks"])
    assert A.apr_step_bins(ctx, ds, [], p["sinks"], DT, 1, 0.3, MAXB) >= 1
