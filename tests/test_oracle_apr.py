"""Pins of the oracle's split/merge pass (no GPU).

Closed forms and invariants from the paper: masses m0/2^l and a factor of
exactly two between levels (Sec. 2.1, rules 4-5); split h scaled by (1/2)^(1/3),
children on opposite sides at r_sep = 0.2 h, tangential to the zone
(Sec. 2.2); merged particle at the pair's centre of mass with its mean velocity
and h scaled by 2^(1/3), leaves of exactly two, at most one spare particle per
level, mass-error bound m0 sum 2^-l < m0 (Sec. 2.3); split before merge, one
level change per pass (Sec. 2.5).  Exact sums use rational arithmetic."""
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
BOX = dict(lo=(0, 0, 0), hi=(1, 1, 1))


def test_splitmix64_reference_vectors(orc):
    for l in open(os.path.join(GOLDEN, "splitmix64_vectors.txt")):
        if l.startswith("#") or not l.strip():
            continue
        seed, *outs = [int(v) for v in l.split()]
        assert [orc.splitmix64(seed, k + 1) for k in range(len(outs))] == outs


def test_cube_root_constants_correctly_rounded():
    # the h factors must be the FP64 values nearest to 2^(-1/3) and 2^(1/3)
    import re
    src = open(os.path.join(os.path.dirname(GOLDEN), "..", "oracle", "apr_oracle.c")).read()
    half = float(re.search(r"ORC_CBRT_HALF ([0-9.]+)", src).group(1))
    two = float(re.search(r"ORC_CBRT_TWO ([0-9.]+)", src).group(1))
    for c, target in ((half, Fr(1, 2)), (two, Fr(2))):
        lo, hi = np.nextafter(c, 0), np.nextafter(c, 10)
        # c^3 is closer to the target than either neighbour's cube
        err = abs(Fr(c) ** 3 - target)
        assert err < abs(Fr(float(lo)) ** 3 - target) and err < abs(Fr(float(hi)) ** 3 - target)


def test_zone_levels_nested_and_strict(orc):
    zones = [dict(c=(0, 0, 0), r=(4.0, 3.0), ell=(1, 2))]
    assert orc.zone_level(0.5, 0, 0, zones) == 2
    assert orc.zone_level(3.0, 0, 0, zones) == 1          # on the inner sphere: outside it
    assert orc.zone_level(3.5, 0, 0, zones) == 1
    assert orc.zone_level(4.0, 0, 0, zones) == 0
    z2 = zones + [dict(c=(3.5, 0, 0), r=(1.0,), ell=(3,))]
    assert orc.zone_level(3.5, 0, 0, z2) == 3             # several zones: max
    assert orc.zone_level(3.5, 0, 0, z2, background=3, derefine=True) == 1  # derefine: min


def test_cylinder_zone_levels(orc):
    # shape 1: cylinders along z through c; the level ignores z, strict radius
    zones = [dict(c=(0.5, 0.5, 7.0), r=(0.3, 0.1), ell=(1, 2), shape=1)]
    for z in (-100.0, 0.0, 7.0, 55.5):
        assert orc.zone_level(0.55, 0.5, z, zones) == 2
        assert orc.zone_level(0.5, 0.75, z, zones) == 1
        assert orc.zone_level(0.8, 0.5, z, zones) == 0     # on the outer cylinder: outside
        assert orc.zone_level(0.5, 0.9, z, zones) == 0
    # in the plane z = c_z a cylinder and a sphere agree
    sph = [dict(zones[0], shape=0)]
    rng = np.random.default_rng(5)
    for x, y in rng.uniform(0.1, 0.9, size=(200, 2)):
        assert orc.zone_level(x, y, 7.0, zones) == orc.zone_level(x, y, 7.0, sph)
    assert orc.zone_level(0.55, 0.5, 7.2, sph) == 1 and orc.zone_level(0.55, 0.5, 7.35, sph) == 0


def test_split_tangential_to_cylinder(orc):
    # a thin periodic box with a cylinder zone: children sit at +-r_sep, at a
    # right angle to the in-plane offset from the axis, whatever their z
    st, p = W.wave_box(nx=16)
    zc = np.array(p["zones"][0]["c"])
    n = st["x"].shape[0]
    out = orc.split_merge(st, p["zones"], step=1, seed=3, r_sep_factor=0.2, nn_cap=0.0,
                          split_mode=0, periodic=True, lo=p["lo"], hi=p["hi"], do_merge=False)
    rxy2 = (st["x"] - zc[0]) ** 2 + (st["y"] - zc[1]) ** 2
    inside = rxy2 < p["zones"][0]["r"][0] ** 2
    par = np.nonzero(inside)[0]
    assert out["n_split"] == par.size > 0
    assert len(set(np.round(st["z"][par], 9))) > 1       # the zone spans several layers
    xp = np.array([st["x"][par], st["y"][par], st["z"][par]])
    d1 = np.array([out["x"][par], out["y"][par], out["z"][par]]) - xp
    v = np.array([xp[0] - zc[0], xp[1] - zc[1], 0.0 * xp[2]])
    cosang = np.sum(d1 * v, axis=0) / (np.linalg.norm(d1, axis=0) * np.linalg.norm(v, axis=0))
    assert np.max(np.abs(cosang)) < 1e-12
    assert _mass_units(out["level"]) == _mass_units(st["level"])
    for k in ("x", "y", "z", "vx"):
        assert _sum_mx(out, k) == _sum_mx(st, k), k


def _small_box(nside=16):
    st, p = W.refine_box(nside=nside)
    p = dict(p, m0=1.0 / nside ** 3)
    return st, p


def _mass_units(level, lmax=8):
    return sum(2 ** (lmax - int(l)) for l in level)


def _sum_mx(st, key, lmax=8):
    return sum(Fr(2 ** (lmax - int(l))) * Fr(float(v)) for l, v in zip(st["level"], st[key]))


def test_split_invariants(orc):
    st, p = _small_box()
    zc = np.array(p["zones"][0]["c"])
    n = st["x"].shape[0]
    out = orc.split_merge(st, p["zones"], step=3, seed=11, r_sep_factor=0.2, nn_cap=0.0,
                          split_mode=0, periodic=True, **BOX, do_merge=False)
    inside = ((st["x"] - zc[0]) ** 2 + (st["y"] - zc[1]) ** 2 + (st["z"] - zc[2]) ** 2) < 0.45 ** 2
    ns = int(inside.sum())
    assert out["n_split"] == ns and out["x"].shape[0] == n + ns
    # mass, momentum and centre of mass exactly conserved
    assert _mass_units(out["level"]) == _mass_units(st["level"])
    for k in ("vx", "vy", "vz", "x", "y", "z"):
        assert _sum_mx(out, k) == _sum_mx(st, k), k
    par = np.nonzero(inside)[0]
    kids = np.arange(n, n + ns)
    assert np.array_equal(out["id"][kids], np.arange(n, n + ns))      # ascending parent order
    assert np.array_equal(out["id"][:n], st["id"])
    assert np.array_equal(out["level"][par], st["level"][par] + 1)
    assert np.array_equal(out["level"][kids], st["level"][par] + 1)
    assert np.array_equal(out["h"][par], st["h"][par] * 0.79370052598409973737585281963615)
    assert np.array_equal(out["h"][kids], out["h"][par])
    for key in ("vx", "vy", "vz", "u"):
        assert np.array_equal(out[key][kids], st[key][par])
    # children at +-r_sep about the parent, tangential to the zone
    xp = np.array([st["x"][par], st["y"][par], st["z"][par]])
    c1 = np.array([out["x"][par], out["y"][par], out["z"][par]])
    c2 = np.array([out["x"][kids], out["y"][kids], out["z"][kids]])
    d1, d2 = c1 - xp, c2 - xp
    rsep = 0.2 * st["h"][par]
    assert np.max(np.abs(np.linalg.norm(d1, axis=0) / rsep - 1)) < 1e-12
    assert np.max(np.abs(np.linalg.norm(d2, axis=0) / rsep - 1)) < 1e-12
    v = xp - zc[:, None]
    cosang = np.sum(d1 * v, axis=0) / (np.linalg.norm(d1, axis=0) * np.linalg.norm(v, axis=0))
    assert np.max(np.abs(cosang)) < 1e-12
    # untouched particles unchanged
    keep = ~inside
    for key in ("x", "y", "z", "h"):
        assert np.array_equal(out[key][:n][keep], st[key][keep])
    # a second pass with the same zone splits each by one more level only
    out2 = orc.split_merge(out, p["zones"], step=4, seed=11, periodic=True, **BOX,
                           do_merge=False)
    assert out2["level"].max() <= 5


def test_split_random_axis_and_cap(orc):
    st, p = _small_box(12)
    n = st["x"].shape[0]
    dnn = np.full(n, 0.01)
    out = orc.split_merge(st, p["zones"], step=0, seed=5, r_sep_factor=0.5, nn_cap=0.35,
                          split_mode=1, periodic=True, **BOX, dnn=dnn, do_merge=False)
    ns = out["n_split"]
    par = np.nonzero(out["level"][:n] != st["level"])[0]
    d = np.array([out["x"][par] - st["x"][par], out["y"][par] - st["y"][par],
                  out["z"][par] - st["z"][par]])
    # 0.5 h = 0.025 > 0.35 * 0.01, so the cap binds everywhere
    assert np.max(np.abs(np.linalg.norm(d, axis=0) / 0.0035 - 1)) < 1e-12
    w = d / np.linalg.norm(d, axis=0)
    assert ns > 500 and np.max(np.abs(w.mean(axis=1))) < 4.0 / np.sqrt(ns)


def test_split_reproducible_and_seeded(orc):
    st, p = _small_box(10)
    a = orc.split_merge(st, p["zones"], step=1, seed=3, periodic=True, **BOX)
    b = orc.split_merge(st, p["zones"], step=1, seed=3, periodic=True, **BOX)
    c = orc.split_merge(st, p["zones"], step=2, seed=3, periodic=True, **BOX)
    assert np.array_equal(a["x"], b["x"]) and not np.array_equal(a["x"], c["x"])


def test_pass_independent_of_array_order(orc):
    # children are numbered by their parents' ids, merges pair by id and
    # position: a permuted copy of the state gives the same particles per id
    st, p = _small_box(10)
    n = st["x"].shape[0]
    st["level"] = np.random.default_rng(2).integers(0, 2, n).astype(np.int8)
    a = orc.split_merge(st, p["zones"], step=1, seed=3, periodic=True, **BOX)
    assert a["n_split"] > 20 and a["n_merged"] > 20
    perm = np.random.default_rng(5).permutation(n)
    sp = {k: (v[perm] if isinstance(v, np.ndarray) else v) for k, v in st.items()}
    b = orc.split_merge(sp, p["zones"], step=1, seed=3, periodic=True, **BOX)
    oa, ob = np.argsort(a["id"]), np.argsort(b["id"])
    assert np.array_equal(a["id"][oa], b["id"][ob])
    for k in ("x", "y", "z", "vx", "vy", "vz", "u", "h", "level"):
        assert np.array_equal(a[k][oa], b[k][ob]), k
    # the children's ids follow their parents' ids
    kids = a["id"] >= n
    parent_id = st["id"][a["origin"][kids]]
    assert np.array_equal(np.argsort(parent_id), np.argsort(a["id"][kids]))
    assert np.array_equal(np.sort(a["id"][kids]), np.arange(n, n + kids.sum()))


def test_capacity_error(orc):
    st, p = _small_box(10)
    with pytest.raises(RuntimeError):
        orc.split_merge(st, p["zones"], step=1, seed=3, periodic=True, **BOX,
                        cap=st["x"].shape[0] + 3)


def test_pair_tree_hand_cases(orc):
    z = np.zeros(6)
    x = np.array([0.05, 0.15, 0.25, 0.35, 0.45, 0.55])
    ids = np.arange(6)
    # 4 on a line: split at the mean into {0,1} {2,3}
    pr = orc.pair_tree(np.arange(4), x, z, z, ids, (0, 0, 0), (1, 1, 1))
    assert sorted(map(tuple, pr.tolist())) == [(0, 1), (2, 3)]
    # 6 on a line: 3 below the mean, 3 above; the tie moves the left side's
    # largest across, giving {0,1} and {2,3,4,5} -> {2,3},{4,5}
    pr = orc.pair_tree(np.arange(6), x, z, z, ids, (0, 0, 0), (1, 1, 1))
    assert sorted(map(tuple, pr.tolist())) == [(0, 1), (2, 3), (4, 5)]
    # 5 candidates: the highest id sits out
    pr = orc.pair_tree(np.arange(5), x, z, z, ids, (0, 0, 0), (1, 1, 1))
    assert 4 not in pr.ravel() and pr.shape == (2, 2)


def test_pair_tree_properties(orc):
    rng = np.random.default_rng(1)
    n = 2000
    x, y, z = rng.uniform(0, 1, (3, n))
    ids = rng.permutation(n).astype(np.int64) * 3 + 7
    cand = np.arange(n)
    pr = orc.pair_tree(cand, x, y, z, ids, (0, 0, 0), (1, 1, 1))
    assert pr.shape == (n // 2, 2) and np.array_equal(np.sort(pr.ravel()), cand)
    # independent of the order candidates are given in
    pr2 = orc.pair_tree(rng.permutation(cand), x, y, z, ids, (0, 0, 0), (1, 1, 1))
    assert sorted(map(tuple, np.sort(pr, 1).tolist())) == sorted(map(tuple, np.sort(pr2, 1).tolist()))
    # pairs are spatial neighbours: mean pair distance below the mean spacing
    dist = np.sqrt((x[pr[:, 0]] - x[pr[:, 1]]) ** 2 + (y[pr[:, 0]] - y[pr[:, 1]]) ** 2 +
                   (z[pr[:, 0]] - z[pr[:, 1]]) ** 2)
    assert dist.mean() < n ** (-1.0 / 3.0)


def test_merge_invariants(orc):
    st, p = _small_box()
    sp = orc.split_merge(st, p["zones"], step=1, seed=2, periodic=True, **BOX, do_merge=False)
    # the zone is gone: every level >= 1 particle is a merge candidate
    out = orc.split_merge(sp, [], step=2, seed=2, periodic=True, **BOX)
    assert out["n_split"] == 0
    levels = np.unique(sp["level"][sp["level"] >= 1])
    counts = {int(l): int((sp["level"] == l).sum()) for l in levels}
    assert out["n_merged"] == sum(c // 2 for c in counts.values())
    assert out["n_spare"] == sum(c % 2 for c in counts.values())
    assert _mass_units(out["level"]) == _mass_units(sp["level"])
    # merged particles sit at their pair's centre of mass: <= 1/2 ulp per merge
    for k in ("x", "vx"):
        err = abs(_sum_mx(out, k) - _sum_mx(sp, k))
        ulp = Fr(float(np.spacing(1.0)))
        assert err <= out["n_merged"] * Fr(2 ** 8) * ulp
    # at most one unmerged particle per level, and the paper's bound on the
    # spare mass, m0 sum_{l=1}^{lmax} 2^-l, stays below m0
    lev_out = dict(zip(out["id"].tolist(), out["level"].tolist()))
    spare_mass = Fr(0)
    for l, c in counts.items():
        ids_l = sp["id"][sp["level"] == l]
        unmerged = [i for i in ids_l.tolist() if lev_out.get(i) == l]
        assert len(unmerged) == c % 2
        spare_mass += len(unmerged) * Fr(1, 2 ** l)
    lmax = int(sp["level"].max())
    assert spare_mass <= sum(Fr(1, 2 ** l) for l in range(1, lmax + 1)) < 1
    # survivors keep their relative order
    pos = {i: k for k, i in enumerate(sp["id"].tolist())}
    assert np.all(np.diff([pos[i] for i in out["id"].tolist()]) > 0)
    # of each merged pair the lower id survives, one level down
    for i, l in lev_out.items():
        assert l in (int(sp["level"][pos[i]]), int(sp["level"][pos[i]]) - 1)


def test_merge_uses_pair_centre_of_mass(orc):
    zones = [dict(c=(0.0, 0.0, 0.0), r=(1.0,), ell=(1,))]
    base = dict(y=np.zeros(2), z=np.zeros(2), vx=np.array([1.0, 3.0]), vy=np.zeros(2),
                vz=np.zeros(2), u=np.array([1.0, 2.0]), h=np.array([0.1, 0.1]),
                level=np.array([1, 1], np.int8), id=np.array([5, 2]), next_id=6)
    kw = dict(step=0, seed=0, lo=(-2, -2, -2), hi=(2, 2, 2), do_split=False)
    inside = orc.split_merge(dict(base, x=np.array([0.9, 1.05])), zones, **kw)
    assert inside["n_merged"] == 0                     # COM 0.975 still in the zone
    out = orc.split_merge(dict(base, x=np.array([0.9, 1.15])), zones, **kw)
    assert out["n_merged"] == 1 and out["x"].shape[0] == 1
    assert out["id"][0] == 2 and out["level"][0] == 0  # lower id kept, one level down
    assert out["x"][0] == (0.9 + 1.15) * 0.5 and out["vx"][0] == 2.0 and out["u"][0] == 1.5
    assert out["h"][0] == 0.1 * 1.2599210498948731647672106072782


def test_pair_tree_degenerate_cuts(orc):
    # quantised coordinates {5,5,5,5,5,5,5,9} (in steps): mean 5.5, floor 5, so
    # nothing lies below the cut; it moves up one step to "<= 5", which holds 7
    # (odd, larger side) -> the largest left particle (id 6) crosses over
    step = 1.0 / 2097152.0
    x = np.array([5, 5, 5, 5, 5, 5, 5, 9], float) * step + 0.25 * step
    z = np.zeros(8)
    ids = np.arange(8)
    pr = orc.pair_tree(np.arange(8), x, z, z, ids, (0, 0, 0), (1, 1, 1))
    got = sorted(map(tuple, np.sort(pr, 1).tolist()))
    # left {0..5} -> split again at its mean (all equal -> by id): {0,1},{2,3},{4,5}
    assert got == [(0, 1), (2, 3), (4, 5), (6, 7)]
    # all particles at one point: split by id order only
    xs = np.full(6, 0.5)
    pr = orc.pair_tree(np.arange(6), xs, xs, xs, np.array([9, 3, 7, 1, 5, 11]), (0, 0, 0),
                       (1, 1, 1))
    assert sorted(map(tuple, np.sort(pr, 1).tolist())) == [(0, 5), (1, 3), (2, 4)]


def test_merge_across_periodic_boundary(orc):
    # Sec. 2.3: the merged particle sits at the pair's centre of mass.  A pair
    # straddling a periodic boundary has it beside the boundary: with the kept
    # particle (lower id) at x = 1/32 and the other at 61/64, the other's
    # minimum image about it is 61/64 - 1 = -3/64, the mean is -1/128, and it
    # wraps to 127/128.  The plain mean would be 63/128, at mid-box; the zone
    # (level 1 inside r = 0.2 of the box centre) makes that difference decide
    # the merge too: 63/128 lies in the zone (no merge), 127/128 outside.
    zones = [dict(c=(0.5, 0.5, 0.5), r=(0.2,), ell=(1,))]
    st = dict(x=np.array([61 / 64, 1 / 32]), y=np.array([0.5, 0.5]), z=np.array([0.5, 0.5]),
              vx=np.array([1.0, 3.0]), vy=np.zeros(2), vz=np.zeros(2), u=np.array([1.0, 2.0]),
              h=np.array([0.01, 0.01]), level=np.array([1, 1], np.int8), id=np.array([5, 2]),
              next_id=6)
    kw = dict(step=0, seed=0, lo=(0, 0, 0), hi=(1, 1, 1), do_split=False)
    out = orc.split_merge(st, zones, periodic=True, **kw)
    assert out["n_merged"] == 1 and out["id"][0] == 2 and out["level"][0] == 0
    assert out["x"][0] == 127 / 128 and out["y"][0] == 0.5 and out["z"][0] == 0.5
    assert out["vx"][0] == 2.0 and out["u"][0] == 1.5
    # the same pair in y and z (kept particle above the boundary this time):
    # mean of 63/64 and 1 + 1/64 is 1, wrapped to 0
    st2 = dict(st, x=np.array([0.25, 0.25]), y=np.array([1 / 64, 63 / 64]),
               z=np.array([1 / 64, 63 / 64]))
    out2 = orc.split_merge(st2, [], periodic=True, **kw)
    assert out2["n_merged"] == 1 and out2["y"][0] == 0.0 and out2["z"][0] == 0.0
    # not periodic: the plain mean, which lies in the zone, so no merge
    assert orc.split_merge(st, zones, periodic=False, **kw)["n_merged"] == 0
