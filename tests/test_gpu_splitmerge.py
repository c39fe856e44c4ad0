"""Split/merge pass on the GPU vs the oracle, slot by slot on identical
inputs: which particles split or merge, the pairing, the survivors' order,
levels, ids, h, velocities and u are bit-exact; positions match to a few
ulp (sin/cos of the split rotation may differ in the last place)."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
import paper_2409_11470_amd as A
import workloads as W
from _gpu import params_for

pytestmark = pytest.mark.gpu


def _ctx(p, **kw):
    d = dict(r_sep_factor=p.get("r_sep_factor", 0.2), nn_cap=p.get("nn_cap", 0.0),
             split_mode=int(p.get("split_mode", 0)), seed=kw.pop("seed", 7))
    d.update(kw)
    return A.Context(params_for(p, "fp64", **d))


def _gpu_pass(st, p, zones, step, flags, seed=7, capacity=None):
    ctx = _ctx(p, seed=seed)
    ds = A.DeviceState.from_numpy(st, capacity=capacity or 2 * st["x"].shape[0] + 8)
    ns, nm, nsp = A.apr_split_merge(ctx, ds, zones, step, flags)
    return ds.to_numpy(), (ns, nm, nsp)


def _orc_pass(st, p, zones, step, flags, seed=7):
    return oracle.split_merge(st, zones, step=step, seed=seed,
                              r_sep_factor=p.get("r_sep_factor", 0.2),
                              nn_cap=p.get("nn_cap", 0.0), split_mode=int(p.get("split_mode", 0)),
                              periodic=p.get("periodic", False), lo=p["lo"], hi=p["hi"],
                              do_split=bool(flags in (0, 1)), do_merge=bool(flags in (0, 2)))


def _compare(g, o, counts):
    ns, nm, nsp = counts
    assert (ns, nm, nsp) == (o["n_split"], o["n_merged"], o["n_spare"])
    n = o["x"].shape[0]
    assert g["x"].shape[0] == n and g["next_id"] == o["next_id"]
    for k in ("id", "level", "h", "vx", "vy", "vz", "u"):
        assert np.array_equal(g[k], o[k]), k
    for k in ("x", "y", "z"):
        scale = np.maximum(np.abs(o[k]), 1.0)
        assert np.max(np.abs(g[k] - o[k]) / scale) < 8 * np.finfo(float).eps, k


@pytest.mark.parametrize("mode", [0, 1])
def test_split_box(mode):
    st, p = W.refine_box(nside=20)
    p = dict(p, m0=1.0 / 20 ** 3, split_mode=mode)
    g, cnt = _gpu_pass(st, p, p["zones"], 5, 1)
    o = _orc_pass(st, p, p["zones"], 5, 1)
    assert cnt[0] > 1000
    _compare(g, o, cnt)


def test_merge_after_zone_moves():
    st, p = W.refine_box(nside=20)
    p = dict(p, m0=1.0 / 20 ** 3)
    sp = _orc_pass(st, p, p["zones"], 1, 1)
    # the zone shrinks: children outside r = 0.3 are merge candidates
    zones = [dict(c=(0.5, 0.5, 0.5), r=(0.3,), ell=(4,))]
    g, cnt = _gpu_pass(sp, p, zones, 2, 2)
    o = _orc_pass(sp, p, zones, 2, 2)
    assert cnt[1] > 100
    _compare(g, o, cnt)


def test_split_and_merge_same_pass():
    st, p = W.refine_box(nside=20)
    p = dict(p, m0=1.0 / 20 ** 3)
    sp = _orc_pass(st, p, p["zones"], 1, 1)
    zones = [dict(c=(0.62, 0.5, 0.45), r=(0.42, 0.2), ell=(4, 5))]
    g, cnt = _gpu_pass(sp, p, zones, 3, 0)
    o = _orc_pass(sp, p, zones, 3, 0)
    assert cnt[0] > 100 and cnt[1] > 100
    _compare(g, o, cnt)


def test_disc_random_split_then_merge():
    st, p = W.planet_disc(n=30000)
    p = dict(p, split_mode=1)
    sp_g, cnt = _gpu_pass(st, p, p["zones"], 0, 0, seed=11)
    sp_o = _orc_pass(st, p, p["zones"], 0, 0, seed=11)
    assert cnt[0] > 100
    _compare(sp_g, sp_o, cnt)
    # the zone moves along the orbit: children left behind merge
    zones = [dict(c=(4.9, 0.9, 0.0), r=(1.0,), ell=(1,))]
    g, cnt = _gpu_pass(sp_o, p, zones, 1, 0, seed=11)
    o = _orc_pass(sp_o, p, zones, 1, 0, seed=11)
    assert cnt[1] > 10
    _compare(g, o, cnt)


def test_merge_many_levels_and_odd_counts():
    # three nested levels from repeated splits, then everything merges back
    st, p = W.refine_box(nside=12)
    p = dict(p, m0=1.0 / 12 ** 3)
    zones = [dict(c=(0.5, 0.5, 0.5), r=(0.45, 0.35, 0.25), ell=(1, 2, 3))]
    st = dict(st, level=np.zeros_like(st["level"]))
    s = st
    for k in range(3):
        s = _orc_pass(s, p, zones, k, 1)
    g, cnt = _gpu_pass(s, p, [], 9, 2)
    o = _orc_pass(s, p, [], 9, 2)
    assert cnt[1] > 100
    _compare(g, o, cnt)


def test_capacity_error_leaves_state():
    st, p = W.refine_box(nside=12)
    p = dict(p, m0=1.0 / 12 ** 3)
    ctx = _ctx(p)
    n = st["x"].shape[0]
    ds = A.DeviceState.from_numpy(st, capacity=n + 5)
    before = ds.to_numpy()
    zarr, nz = A.make_zones(p["zones"])
    cs = ds.cstate()
    ns, nm, nsp = C.c_int64(), C.c_int64(), C.c_int64()
    rc = A.lib().apr_split_merge(ctx.ptr, C.byref(cs), zarr, nz, 1, 0, C.byref(ns), C.byref(nm),
                                 C.byref(nsp))
    assert rc == A.APR_ERR_CAPACITY and ns.value > n + 5 and cs.n == n
    after = ds.to_numpy()
    for k in ("x", "h", "level", "id"):
        assert np.array_equal(before[k], after[k])


def test_merge_pairs_across_periodic_boundary():
    # four level-1 pairs, each straddling the x boundary of a periodic box
    # (minimum-image separation 0.3-0.4, plain separation above half the box),
    # the pairs at the corners (y, z) in {0.02, 0.98}^2, so that the tree cuts
    # y and z first and pairs them as built.  A small level-1 sphere sits on
    # each pair's plain mean (x near 0.5): only a centre of mass taken across
    # the boundary lies outside it, so every pair merges
    rng = np.random.default_rng(2409114791)
    g = 4
    xa = 0.15 + 0.05 * rng.random(g)
    xb = 0.80 + 0.05 * rng.random(g)
    y = np.array([0.02, 0.02, 0.98, 0.98]) + 1e-3 * rng.random(g)
    z = np.array([0.02, 0.98, 0.02, 0.98]) + 1e-3 * rng.random(g)
    n = 2 * g
    st = dict(x=np.concatenate([xa, xb]), y=np.concatenate([y, y]), z=np.concatenate([z, z]),
              vx=rng.standard_normal(n), vy=rng.standard_normal(n), vz=rng.standard_normal(n),
              u=1.0 + rng.random(n), h=np.full(n, 0.02), level=np.ones(n, np.int8),
              id=rng.permutation(n).astype(np.int64), next_id=n)
    p = dict(lo=(0, 0, 0), hi=(1, 1, 1), periodic=True, m0=1.0 / 4096)
    zones = [dict(c=(0.5 * (xa[k] + xb[k]), y[k], z[k]), r=(0.1,), ell=(1,)) for k in range(g)]
    gp, cnt = _gpu_pass(st, p, zones, 0, 2)
    o = _orc_pass(st, p, zones, 0, 2)
    assert cnt[1] == g
    _compare(gp, o, cnt)
    assert np.all((o["x"] < 0.1) | (o["x"] >= 0.9))


@pytest.mark.parametrize("nlev1", [2, 3, 4, 5, 6, 40, 255, 600, 1023, 1024, 1025, 1026, 1500])
def test_merge_tree_sizes(nlev1):
    """n randomly chosen level-1 particles of the box and no zone: every pair
    merges.  The candidates are ordered by id in one workgroup up to 1024 and
    by radix sort beyond, and the pairing tree of the n (n - 1 when odd) is
    built in one workgroup up to 1024 elements and depth by depth beyond;
    all against the oracle."""
    st, p = W.refine_box(nside=12)
    p = dict(p, m0=1.0 / 12 ** 3)
    rng = np.random.default_rng(5)
    lev = np.zeros_like(st["level"])
    lev[rng.choice(st["x"].shape[0], nlev1, replace=False)] = 1
    st = dict(st, level=lev)
    g, cnt = _gpu_pass(st, p, [], 3, 2)
    o = _orc_pass(st, p, [], 3, 2)
    assert cnt[1] == nlev1 // 2 and cnt[2] == nlev1 % 2
    _compare(g, o, cnt)
