"""Pins of the oracle's individual timesteps (paper Sec. 2.5; no GPU)."""
import numpy as np
import pytest

import workloads as W


def _phys(p):
    return dict(m0=p["m0"], eos=p["eos"], cs0=p.get("cs0", 1.0), q_cs=p.get("q_cs", 0.25),
                r_ref=p.get("r_ref", 1.0), gamma=p.get("gamma", 5.0 / 3.0),
                alpha=p.get("alpha", 1.0), beta=p.get("beta", 2.0), hfact=p.get("hfact", 1.2),
                periodic=p.get("periodic", False), lo=p.get("lo", (0, 0, 0)),
                hi=p.get("hi", (1, 1, 1)))


def _global_step(orc, st, phys, zones, dt, key, sm):
    """One kick-drift-kick step of the whole set with a split/merge pass, from
    the oracle's functions (the order of a step, Sec. 2.6)."""
    box = dict(periodic=phys["periodic"], lo=phys["lo"], hi=phys["hi"])
    adiab = phys["eos"] == 2
    orc.kick(st["vx"], st["vy"], st["vz"], st["u"] if adiab else None, st["ax"], st["ay"],
             st["az"], st["dudt"] if adiab else None, 0.5 * dt)
    orc.drift(st["x"], st["y"], st["z"], st["vx"], st["vy"], st["vz"], dt, **box)
    if zones:
        out = orc.split_merge(st, zones, step=key, dnn=st["dnn"], **sm, **box)
        o = out["origin"]
        new = {k: out[k] for k in ("x", "y", "z", "vx", "vy", "vz", "u", "h", "level", "id",
                                   "next_id")}
        for k in ("rho", "omega", "ax", "ay", "az", "dudt", "vsig", "dnn", "bin"):
            new[k] = st[k][o].copy()
        st = new
    orc.accel_bins(st, **phys)
    orc.kick(st["vx"], st["vy"], st["vz"], st["u"] if adiab else None, st["ax"], st["ay"],
             st["az"], st["dudt"] if adiab else None, 0.5 * dt)
    return st


def _same(a, b, keys=("x", "y", "z", "vx", "vy", "vz", "u", "h")):
    oa, ob = np.argsort(a["id"]), np.argsort(b["id"])
    assert np.array_equal(a["id"][oa], b["id"][ob])
    for k in keys:
        assert np.array_equal(a[k][oa], b[k][ob]), k


def test_bin_zero_is_the_global_step(orc):
    st, p = W.wave_box(nx=16)
    phys = _phys(p)
    sm = dict(seed=3, r_sep_factor=0.2, nn_cap=0.35, split_mode=0)
    orc.accel_bins(st, **phys)
    st["bin"] = np.zeros(st["x"].shape[0], np.int8)
    dt = 0.25 * float(st["h"].min())
    a = orc.step_bins(st, zones=p["zones"], dt_max=dt, step=5, max_bin=0, **sm, **phys)
    b = _global_step(orc, {k: (v.copy() if isinstance(v, np.ndarray) else v)
                           for k, v in st.items()}, phys, p["zones"], dt, 5 * 4096, sm)
    assert a["x"].shape[0] > st["x"].shape[0]
    _same(a, b)


def test_uniform_finest_bin_is_substepping(orc):
    # a lattice (uniform Courant limit) with dt_max four times that limit:
    # every particle sits in bin 2 throughout, i.e. four global steps
    st, p = W.lattice_box(nside=10)
    st = dict(st, u=np.zeros_like(st["x"]))
    p = dict(p, m0=1e-3)
    phys = _phys(p)
    orc.accel_bins(st, **phys)
    dtc = 0.3 * st["h"] / st["vsig"]
    dtm = 3.9 * dtc.min()
    assert dtm <= 4 * dtc.min() and dtm > 2 * dtc.max()
    st["bin"] = orc.courant_bin(st["h"], st["vsig"], dt_max=dtm, c_cfl=0.3, max_bin=2)
    assert np.all(st["bin"] == 2)
    a = orc.step_bins(st, zones=[], dt_max=dtm, step=0, max_bin=2, **phys)
    b = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()}
    for _ in range(4):
        b = _global_step(orc, b, phys, [], np.ldexp(dtm, -2), 0, {})
    _same(a, b)
    assert np.all(a["bin"] == 2)


def test_split_only_active_and_new_particles_finest(orc):
    st, p = W.wave_box(nx=16)
    phys = _phys(p)
    orc.accel_bins(st, **phys)
    n = st["x"].shape[0]
    rng = np.random.default_rng(4)
    st["bin"] = rng.integers(0, 2, n).astype(np.int8)       # bins 0 and 1: K = 1
    z = p["zones"][0]
    inside = (st["x"] - z["c"][0]) ** 2 + (st["y"] - z["c"][1]) ** 2 < z["r"][0] ** 2
    dt = 0.5 * float(st["h"].min())
    a = orc.step_bins(st, zones=p["zones"], dt_max=dt, step=1, max_bin=1, seed=3,
                      r_sep_factor=0.2, nn_cap=0.35, split_mode=0, **phys)
    kids = a["id"] >= n
    assert kids.sum() == inside.sum()
    # bin-1 parents are active at the end of substep 0, bin-0 parents only at
    # the end of substep 1: by the end of the step every parent has split once
    par1 = np.sort(st["id"][inside & (st["bin"] == 1)])
    par0 = np.sort(st["id"][inside & (st["bin"] == 0)])
    assert par1.size > 0 and par0.size > 0
    ids = np.sort(a["id"][kids])
    assert np.array_equal(ids, np.arange(n, n + inside.sum()))
    # every particle the pass made or kept sits in the finest bin
    made = np.isin(a["id"], np.concatenate([par1, par0])) | kids
    assert np.all(a["bin"][made] == 1)


def test_pass_examines_active_particles_only(orc):
    st, p = W.wave_box(nx=16)
    n = st["x"].shape[0]
    box = dict(periodic=True, lo=p["lo"], hi=p["hi"])
    act = np.random.default_rng(6).random(n) < 0.5
    z = p["zones"][0]
    inside = (st["x"] - z["c"][0]) ** 2 + (st["y"] - z["c"][1]) ** 2 < z["r"][0] ** 2
    out = orc.split_merge(st, p["zones"], step=1, seed=3, r_sep_factor=0.2, nn_cap=0.0,
                          active=act, do_merge=False, **box)
    assert out["n_split"] == (inside & act).sum() > 0
    split = out["level"][:n] == 1
    assert np.array_equal(split, inside & act)
    assert np.array_equal(out["origin"][n:], np.nonzero(inside & act)[0])
    assert np.all(out["changed"][n:]) and np.array_equal(out["changed"][:n], inside & act)
    # merging: level-1 particles outside every zone pair among the active ones
    lv = dict(st, level=np.ones(n, np.int8))
    far = [dict(c=(0.5, 0.5, 0.0), r=(1e-9,), ell=(1,), shape=1)]
    m_all = orc.split_merge(lv, far, step=1, seed=3, do_split=False, **box)
    m_act = orc.split_merge(lv, far, step=1, seed=3, do_split=False, active=act, **box)
    assert m_all["n_merged"] == n // 2
    assert m_act["n_merged"] == act.sum() // 2
    gone = np.setdiff1d(lv["id"], m_act["id"])
    assert np.all(act[gone])


def test_bins_refine_past_k_only_at_the_step_end(orc):
    # every particle starts in bin 0 (K = 0, one substep) while the Courant
    # limit asks for bin 2: at the end of the step, where every particle is
    # synchronised, the bin follows the limit up to max_bin
    st, p = W.lattice_box(nside=10)
    st = dict(st, u=np.zeros_like(st["x"]))
    p = dict(p, m0=1e-3)
    phys = _phys(p)
    orc.accel_bins(st, **phys)
    dtc = 0.3 * st["h"] / st["vsig"]
    dtm = 3.9 * dtc.min()
    st["bin"] = np.zeros(st["x"].shape[0], np.int8)
    a = orc.step_bins(st, zones=[], dt_max=dtm, step=0, max_bin=4, **phys)
    assert np.all(a["bin"] == 2)
    b = orc.step_bins(st, zones=[], dt_max=dtm, step=0, max_bin=1, **phys)
    assert np.all(b["bin"] == 1)
