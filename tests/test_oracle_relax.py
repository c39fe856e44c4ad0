"""Pins of the oracle's relaxing (paper Sec. 2.4) and of the interpolation it
uses (no GPU)."""
import numpy as np
import pytest

import workloads as W

BOX1 = dict(periodic=True, lo=(0, 0, 0), hi=(1, 1, 1))


def _lattice(orc, kernel, hfact):
    st, p = W.lattice_box(nside=8)
    d = orc.density(st["x"], st["y"], st["z"], st["level"], st["h"], m0=p["m0"], tol=1e-14,
                    max_iter=60, hfact=hfact, kernel=kernel, **BOX1)
    assert d["failures"] == 0
    return st, p, d


@pytest.mark.parametrize("kernel,hfact", [(0, 1.2), (1, 1.3)])
def test_interp_of_constant_field_on_converged_lattice(orc, kernel, hfact):
    # with rho the converged density sum, sum_b (m/rho) W(x_a - x_b, h) = 1 at
    # every lattice site, so a constant field comes back exactly
    st, p, d = _lattice(orc, kernel, hfact)
    n = st["x"].shape[0]
    A = np.array([1.5, -2.0, 0.25])
    q = (p["m0"] / d["rho"])[None, :] * A[:, None]
    out = orc.interp(st["x"], st["y"], st["z"], st["x"], st["y"], st["z"], d["h"], q,
                     kernel=kernel, **BOX1)
    assert np.max(np.abs(out - A[:, None] * np.ones(n))) < 1e-12


def test_interp_single_particle_support_and_wrap(orc):
    r = np.array([0.5]), np.array([0.5]), np.array([0.5])
    h = np.array([0.1])
    q = np.array([[2.0], [0.0], [-1.0]])
    # inside the support, on its edge (strict: nothing) and beyond it
    for dist, expect in ((0.07, orc.w(0.07, 0.1)), (0.2, 0.0), (0.25, 0.0)):
        o = orc.interp([0.5 + dist], [0.5], [0.5], *r, h, q, **BOX1)
        tol = 1e-12 * max(expect, 1e-30)  # 0.5 + dist - 0.5 is dist to rounding
        assert abs(o[0, 0] - 2.0 * expect) <= 2 * tol + 1e-40
        assert abs(o[2, 0] + expect) <= tol + 1e-40
    # through the periodic boundary: x = 0.02 sees a particle at 0.97 at 0.05
    o = orc.interp([0.02], [0.5], [0.5], [0.97], [0.5], [0.5], h, q, **BOX1)
    assert abs(o[0, 0] / (2.0 * orc.w(0.05, 0.1)) - 1.0) < 1e-12
    o = orc.interp([0.02], [0.5], [0.5], [0.97], [0.5], [0.5], h, q, periodic=False)
    assert o[0, 0] == 0.0


def _refined_wave(orc):
    st, p = W.wave_box(nx=16)
    box = dict(periodic=True, lo=p["lo"], hi=p["hi"])
    d = orc.density(st["x"], st["y"], st["z"], st["level"], st["h"], m0=p["m0"], tol=1e-12,
                    max_iter=60, **box)
    ref = dict(st, h=d["h"])
    f = orc.forces(ref["x"], ref["y"], ref["z"], ref["vx"], ref["vy"], ref["vz"], ref["u"],
                   ref["level"], d["h"], d["rho"], d["omega"], m0=p["m0"], eos=2,
                   gamma=p["gamma"], **box)
    new = orc.split_merge(ref, p["zones"], step=1, seed=7, r_sep_factor=0.2, nn_cap=0.35,
                          split_mode=0, do_merge=False, dnn=d["dnn"], **box)
    kw = dict(m0=p["m0"], eos=2, gamma=p["gamma"], **box)
    return ref, new, d["rho"], np.array([f["ax"], f["ay"], f["az"]]), kw


def test_relax_moves_only_introduced_particles(orc):
    ref, new, rho, a, kw = _refined_wave(orc)
    n0 = ref["x"].shape[0]
    moved = new["level"] != np.concatenate([ref["level"], np.full(new["n_split"], -1)])
    moved[n0:] = True
    x0 = {k: new[k].copy() for k in ("x", "y", "z")}
    ns, kes = orc.relax(new, ref, rho, a, max_shuffles=3, ke_frac=0.0, **kw)
    assert ns == 3 and len(kes) == 3 and kes[0] > 0
    d = np.sqrt(sum((new[k] - x0[k]) ** 2 for k in ("x", "y", "z")))
    assert np.all(d[~moved] == 0.0) and np.all(d[moved] > 0.0)
    assert kes[2] < kes[1] < kes[0]            # the shuffles settle (Sec. 2.4)


def test_relax_nothing_introduced_stops_at_once(orc):
    ref, new, rho, a, kw = _refined_wave(orc)
    same = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in ref.items()}
    ns, kes = orc.relax(same, ref, rho, a, **kw)
    assert ns == 1 and kes == [0.0]
    for k in ("x", "y", "z"):
        assert np.array_equal(same[k], ref[k])


def test_relax_shift_capped_at_h(orc):
    # an enormous reference acceleration: every shuffled particle moves h
    ref, new, rho, a, kw = _refined_wave(orc)
    x0 = {k: new[k].copy() for k in ("x", "y", "z")}
    big = np.zeros_like(a)
    big[1] = 1e12
    ns, kes = orc.relax(new, ref, rho, big, max_shuffles=1, **kw)
    L = np.asarray(kw["hi"], float)
    d = np.array([new[k] - x0[k] for k in ("x", "y", "z")])
    d -= L[:, None] * np.round(d / L[:, None])
    ln = np.sqrt((d * d).sum(0))
    sel = ln > 0
    assert sel.sum() >= 2 * new["n_split"]
    assert np.max(np.abs(ln[sel] / new["h"][sel] - 1.0)) < 1e-9
    assert np.all(d[1, sel] < 0)               # against the reference acceleration


def test_relax_stop_rule(orc):
    ref, new, rho, a, kw = _refined_wave(orc)
    n1, k1 = orc.relax({k: (v.copy() if isinstance(v, np.ndarray) else v)
                        for k, v in new.items()}, ref, rho, a, ke_frac=0.95, **kw)
    # stops at the first shuffle whose KE is at most 95% of the first one's
    assert k1[-1] <= 0.95 * k1[0] and all(k > 0.95 * k1[0] for k in k1[1:-1])
    n2, k2 = orc.relax(new, ref, rho, a, max_shuffles=4, ke_frac=0.0, **kw)
    # the same shuffles up to where the first run stopped
    m = min(n1, 4)
    assert n2 == 4 and k2[:m] == k1[:m]
