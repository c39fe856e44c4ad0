"""Parity at the full sizes of the disc and refinement workloads, in the launch
configuration the benchmark uses: the 1M-particle planet disc, the 8M-particle
circumbinary disc (three masses) and the refined box (262144 particles of
which about 1e5 split).  Density and forces are compared on sampled targets
the oracle solves exactly (ball samples with complete source sets); the split
and merge passes are compared slot by slot; the adjoint's split-separation
derivative against central differences of the oracle on a sampled loss."""
import numpy as np
import pytest
import torch

import oracle
import paper_2409_11470_amd as A
import workloads as W
from _gpu import exact_counts, gpu_density, gpu_forces, oracle_balls, params_for

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-5, "fp32": 1e-3}


def _rel(a, b):
    return float(np.max(np.abs(a - b) / np.abs(b)))


def _check(g, gf, tg, od, of, prec):
    assert od["failures"] == 0 and g["failures"] == 0
    for k in ("h", "rho", "omega"):
        assert _rel(g[k][tg], od[k]) < TOL[prec], k
    da = np.sqrt(sum((gf[k][tg] - of[k]) ** 2 for k in ("ax", "ay", "az")))
    assert np.max(da / of["anorm"]) < TOL[prec]
    assert np.max(np.abs(gf["dudt"][tg] - of["dudt"]) / np.maximum(of["unorm"], 1e-300)) \
        < TOL[prec]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_planet_disc_1M_sampled(prec):
    st, p = W.planet_disc()
    g, ctx, ds, (rho, om) = gpu_density(st, p, prec)
    gf = gpu_forces(ctx, ds, rho, om)
    tg, od, of = oracle_balls(st, p, 6, 48, seed=21)
    _check(g, gf, tg, od, of, prec)
    # the density kernel's own neighbour counts at the h it returned, exactly
    # (the disc has cells whose candidates span several staging windows, where
    # an accepted Halley step keeps the pass's count only when no pair lies
    # between the supports)
    assert np.array_equal(g["nneigh"][tg], exact_counts(st, p, tg, g["h"]))


def _final_state(ctx, ds):
    """Density and hydro forces of the state as a step left it (cells built
    again), all in storage order: (state arrays, density dict, forces dict)."""
    A.apr_build_cells(ctx, ds)
    rho = torch.zeros(ds.n, dtype=ctx.dtype, device="cuda")
    om = torch.zeros_like(rho)
    A.apr_density(ctx, ds, rho, om)
    f = {k: torch.zeros_like(rho) for k in ("ax", "ay", "az", "dudt", "vsig")}
    A.apr_forces(ctx, ds, rho, om, f["ax"], f["ay"], f["az"], f["dudt"], f["vsig"])
    assert A.apr_sync_status(ctx) == 0
    s = ds.to_numpy()
    g = dict(h=s["h"], rho=rho.double().cpu().numpy(), omega=om.double().cpu().numpy(),
             failures=0)
    return s, g, {k: v.double().cpu().numpy() for k, v in f.items()}


def test_shock_box_262k_20_steps_fp32():
    # The benchmarked sequence at its full size: the 64^3 jittered box with its
    # two states, 20 leapfrog steps in the FP32 form at dt = 0.3 min(h / v_sig)
    # of t = 0; at the final state, the density and hydro forces of sampled
    # balls (four about the interface x = 0.5, four anywhere) against the
    # oracle at the GPU's own positions.
    st, p = W.shock_box()
    ctx = A.Context(params_for(p, "fp32"))
    ds = A.DeviceState.from_numpy(st)
    A.apr_accel(ctx, ds)
    dt = A.apr_timestep(ctx, ds, 0.3)
    for k in range(20):
        A.apr_step(ctx, ds, [], [], dt, k)
    assert A.apr_sync_status(ctx) == 0
    s, g, gf = _final_state(ctx, ds)
    del ctx, ds
    n = s["x"].shape[0]
    rng = np.random.default_rng(24)
    near = np.nonzero(np.abs(s["x"] - 0.5) < 0.02)[0]
    centres = np.concatenate([rng.choice(near, 4, replace=False),
                              rng.choice(n, 4, replace=False)])
    tg, od, of = oracle_balls(s, p, 8, 48, seed=24, centres=centres)
    _check(g, gf, tg, od, of, "fp32")


def test_planet_disc_1M_10_steps_with_refinement():
    # The 1M disc's ten leapfrog steps with its refinement sphere (r = 1 about
    # (5, 0, 0), random split axes, r_sep = 0.5 h, the sink at the origin), as
    # the benchmark runs them (FP32 form, dt = 2e-3): particles split as they
    # enter the sphere and pairs merge as they leave, every step.  At any size:
    # no failure, the mass in units of the smallest particle unchanged, ids
    # unique, every particle well inside the sphere at its level and none above
    # it.  At the final state: the density and hydro forces of sampled balls
    # against the oracle at the GPU's own positions.
    st, p = W.planet_disc()
    ctx = A.Context(params_for(p, "fp32", r_sep_factor=p["r_sep_factor"], nn_cap=p["nn_cap"],
                               split_mode=int(p["split_mode"]), seed=3,
                               G=float(p.get("G", 1.0))))
    ds = A.DeviceState.from_numpy(st, capacity=st["x"].shape[0] * 5 // 4)
    units = lambda lv: int(np.sum(2 ** (8 - lv.astype(np.int64))))
    u0 = units(st["level"])
    A.apr_accel(ctx, ds, p["sinks"])
    for k in range(10):
        A.apr_step(ctx, ds, p["zones"], p["sinks"], 2e-3, k)
    assert A.apr_sync_status(ctx) == 0
    fin = ds.to_numpy()
    assert units(fin["level"]) == u0
    assert fin["x"].shape[0] > st["x"].shape[0]
    assert np.unique(fin["id"]).shape[0] == fin["id"].shape[0]
    c = np.array(p["zones"][0]["c"])
    r2 = (fin["x"] - c[0]) ** 2 + (fin["y"] - c[1]) ** 2 + (fin["z"] - c[2]) ** 2
    assert np.all(fin["level"][r2 < 0.9 ** 2] == 1) and np.all(fin["level"] <= 1)
    s, g, gf = _final_state(ctx, ds)
    del ctx, ds
    n = s["x"].shape[0]
    # three balls anywhere, three about children (both masses in their reach)
    rng = np.random.default_rng(22)
    centres = np.concatenate([rng.choice(n, 3, replace=False),
                              rng.choice(np.nonzero(s["level"] == 1)[0], 3, replace=False)])
    tg, od, of = oracle_balls(s, p, 6, 48, seed=22, centres=centres)
    _check(g, gf, tg, od, of, "fp32")


@pytest.fixture(scope="module")
def cb_disc():
    return W.circumbinary_disc()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_circumbinary_8M_sampled(cb_disc, prec):
    st, p = cb_disc
    g, ctx, ds, (rho, om) = gpu_density(st, p, prec)
    gf = gpu_forces(ctx, ds, rho, om)
    del ctx, ds, rho, om
    torch.cuda.empty_cache()
    # two balls centred on particles of each level (0 outer disc, 1 and 2
    # the refined rings about the binary)
    rng = np.random.default_rng(22)
    centres = np.concatenate([rng.choice(np.nonzero(st["level"] == l)[0], 2, replace=False)
                              for l in (0, 1, 2)])
    tg, od, of = oracle_balls(st, p, 6, 48, seed=22, centres=centres)
    assert set(np.unique(st["level"][tg])) == {0, 1, 2}
    _check(g, gf, tg, od, of, prec)


def _orc_pass(st, p, zones, step, flags, seed=7):
    return oracle.split_merge(st, zones, step=step, seed=seed,
                              r_sep_factor=p.get("r_sep_factor", 0.2),
                              nn_cap=p.get("nn_cap", 0.0), split_mode=int(p.get("split_mode", 0)),
                              periodic=p.get("periodic", False), lo=p["lo"], hi=p["hi"],
                              do_split=bool(flags in (0, 1)), do_merge=bool(flags in (0, 2)))


def _gpu_pass(st, p, zones, step, flags, seed=7):
    ctx = A.Context(params_for(p, "fp64", r_sep_factor=p.get("r_sep_factor", 0.2),
                               nn_cap=p.get("nn_cap", 0.0),
                               split_mode=int(p.get("split_mode", 0)), seed=seed))
    ds = A.DeviceState.from_numpy(st, capacity=2 * st["x"].shape[0] + 8)
    cnt = A.apr_split_merge(ctx, ds, zones, step, flags)
    return ds.to_numpy(), cnt


def _compare(g, o, cnt):
    assert tuple(cnt) == (o["n_split"], o["n_merged"], o["n_spare"])
    assert g["x"].shape[0] == o["x"].shape[0] and g["next_id"] == o["next_id"]
    for k in ("id", "level", "h", "vx", "vy", "vz", "u"):
        assert np.array_equal(g[k], o[k]), k
    for k in ("x", "y", "z"):
        scale = np.maximum(np.abs(o[k]), 1.0)
        assert np.max(np.abs(g[k] - o[k]) / scale) < 8 * np.finfo(float).eps, k


def test_refine_box_full_split():
    st, p = W.refine_box()
    g, cnt = _gpu_pass(st, p, p["zones"], 3, 1)
    o = _orc_pass(st, p, p["zones"], 3, 1)
    assert cnt[0] > 90000
    _compare(g, o, cnt)


def test_circumbinary_8M_merge(cb_disc):
    # shrink both zones: level-2 pairs between r = 2.5 and 3, level-1 pairs
    # between 3.5 and 4 merge; 1.4M level-2 and 0.7M level-1 candidates
    st, p = cb_disc
    zones = [dict(c=(0.0, 0.0, 0.0), r=(3.5, 2.5), ell=(1, 2))]
    g, cnt = _gpu_pass(st, p, zones, 4, 2)
    o = _orc_pass(st, p, zones, 4, 2)
    assert cnt[1] > 100000
    _compare(g, o, cnt)


# ------------------------------------------------------------------ adjoint
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_refine_box_split_separation_gradient(prec):
    """The refined box after its split pass (about 362k particles); loss over
    64 sampled child pairs, L = sum (rho_c - rho_parent)^2, as a function of
    the separation factor s (children at centre +- s h w).  The adjoint's dL/ds
    (all particles in the forward) vs central differences of the oracle."""
    st, p = W.refine_box()
    n0 = st["x"].shape[0]
    s1 = _orc_pass(st, p, p["zones"], 3, 1)
    n1 = s1["x"].shape[0]
    split = np.nonzero(s1["level"][:n0] > st["level"])[0]
    pb_all = n0 + np.arange(n1 - n0)
    X1 = np.stack([s1["x"], s1["y"], s1["z"]], 1)
    dX = X1[split] - X1[pb_all]
    dX -= np.round(dX)  # periodic unit box
    e = dX / (2 * 0.2)
    centre = X1[pb_all] + 0.5 * dX
    rng = np.random.default_rng(31)
    pick = rng.choice(split.size, 64, replace=False)
    pa, pb = split[pick], pb_all[pick]
    # the unsplit parents' densities (constants of the loss)
    pd = oracle.density(st["x"], st["y"], st["z"], st["level"], st["h"][split[pick]],
                        m0=p["m0"], tol=1e-14, max_iter=100, periodic=True, targets=split[pick])
    rho_ref = pd["rho"]

    def positions(s):
        X = X1.copy()
        X[split] = centre + s * e
        X[pb_all] = centre - s * e
        return X - np.floor(X)

    # oracle: densities of the 128 sampled children over the sources near them
    tg = np.concatenate([pa, pb])

    def c_loss(s):
        X = positions(s)
        st2 = dict(s1, x=X[:, 0], y=X[:, 1], z=X[:, 2])
        d = pos_density(st2, tg)
        return float(np.sum((d[:64] - rho_ref) ** 2 + (d[64:] - rho_ref) ** 2))

    def pos_density(st2, targets):
        P = np.stack([st2["x"], st2["y"], st2["z"]], 1)
        hm = 2.0 * float(np.max(st2["h"]))
        src = np.zeros(P.shape[0], bool)
        for t in targets:
            d = P - P[t]
            d -= np.round(d)
            src |= (d * d).sum(1) < (2.2 * hm) ** 2
        S = np.nonzero(src)[0]
        loc = np.full(P.shape[0], -1)
        loc[S] = np.arange(S.size)
        o = oracle.density(P[S, 0], P[S, 1], P[S, 2], st2["level"][S], st2["h"][targets],
                           m0=p["m0"], tol=1e-14, max_iter=100, periodic=True,
                           targets=loc[targets])
        assert o["failures"] == 0 and np.all(o["h"] < hm)
        return o["rho"]

    s0, eps = 0.2, 1e-6
    fd = (c_loss(s0 + eps) - c_loss(s0 - eps)) / (2 * eps)

    ctx = A.Context(params_for(p, prec))
    ds = A.DeviceState.from_numpy(s1)
    s = torch.tensor(s0, dtype=torch.float64, device="cuda", requires_grad=True)
    cen = torch.tensor(centre, device="cuda")
    et = torch.tensor(e, device="cuda")
    ia = torch.as_tensor(split, device="cuda")
    ib = torch.as_tensor(pb_all, device="cuda")
    X = torch.tensor(X1, device="cuda")
    X = X.index_put((ia,), cen + s * et).index_put((ib,), cen - s * et)
    X = X - torch.floor(X).detach()
    rho, *_ = A.apr_sums(ctx, ds, X[:, 0].contiguous(), X[:, 1].contiguous(),
                         X[:, 2].contiguous())
    ref = torch.tensor(rho_ref, device="cuda")
    ta, tb = torch.as_tensor(pa, device="cuda"), torch.as_tensor(pb, device="cuda")
    loss = ((rho.double()[ta] - ref) ** 2 + (rho.double()[tb] - ref) ** 2).sum()
    loss.backward()
    an = float(s.grad)
    print(f"full-size r_sep gradient {prec}: {an:.10e} fd {fd:.10e}")
    assert abs(an - fd) < (1e-4 if prec == "fp64" else 1e-3) * abs(fd), (an, fd)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("level", [0, 1, 2])
def test_circumbinary_8M_vjp_sampled(cb_disc, prec, level):
    # the adjoint on the 8M disc: one ball centred on a particle of each level
    # (masses m, m/2, m/4), cotangents on its 16 targets, gradients over all
    # 8M particles against the dense gradient oracle on the ball's dependency
    # set; gates 1e-6 (FP64) and 1e-3 (FP32) of the max-norm
    from _gpu import ball_vjp_check
    st, p = cb_disc
    rng = np.random.default_rng(2409114705 + level)
    centre = int(rng.choice(np.nonzero(st["level"] == level)[0]))
    ball_vjp_check(("circumbinary", level), st, p, prec, centre, seed=level,
                   gtol={"fp64": 1e-6, "fp32": 1e-3}[prec])


@pytest.fixture(scope="module")
def refined_box():
    # the split pass's result, given a seeded velocity field (N(0, 0.1) per
    # component, a tenth of the sound speed) so that du/dt and the viscosity
    # take part in the adjoint
    st, p = W.refine_box()
    s1 = _orc_pass(st, p, p["zones"], 3, 1)
    v = np.random.default_rng(41).normal(0.0, 0.1, size=(3, s1["x"].shape[0]))
    return dict(s1, vx=v[0], vy=v[1], vz=v[2]), p


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("level", [1, 4])
def test_refine_box_vjp_sampled(refined_box, prec, level):
    # the adjoint on the refined box after its split pass (362k particles,
    # levels 0, 1, 3, 4, in motion): one ball on the sphere's edge about a child of each
    # split level, so the ball holds children and their unsplit neighbours;
    # x-bar and m-bar over all particles against the dense gradient oracle on
    # the ball's dependency set; gates 1e-6 (FP64) and 1e-3 (FP32) of the
    # max-norm
    from _gpu import ball_vjp_check
    s1, p = refined_box
    z = p["zones"][0]
    r = np.sqrt((s1["x"] - z["c"][0]) ** 2 + (s1["y"] - z["c"][1]) ** 2 +
                (s1["z"] - z["c"][2]) ** 2)
    ch = np.nonzero(s1["level"] == level)[0]
    centre = int(ch[np.argmin(np.abs(r[ch] - z["r"][0]))])
    ball_vjp_check(("refined_box", level), s1, p, prec, centre, seed=40 + level,
                   gtol={"fp64": 1e-6, "fp32": 1e-3}[prec])


def test_beyond_16M_particles_scans_cells_density():
    # 272^3 = 20.1M particles (the benchmarked box's shape): the cell build,
    # the density and the neighbour export run scans of more than 4096 tiles
    # of 4096 elements (the recursive level of the scan).  The export's
    # offsets must be the exact prefix sums of its counts, the density
    # kernel's own neighbour count must equal the export's (FP64 predicate)
    # for every particle, and sampled densities must match the oracle.
    import ctypes as C
    nside = 272
    st, p = W.shock_box(nside=nside)
    p = dict(p, m0=1.0 / nside ** 3)
    n = st["x"].shape[0]
    assert n > 4096 * 4096
    g, ctx, ds, (rho, om) = gpu_density(st, p, "fp32")
    assert g["failures"] == 0
    cs = ds.cstate()
    counts = torch.zeros(n, dtype=torch.int64, device="cuda")
    offs = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    total = C.c_int64()
    hd = ds["h"].contiguous()
    rc = A.lib().apr_neighbours(ctx.ptr, C.byref(cs), C.c_void_p(hd.data_ptr()), 0,
                                C.c_void_p(counts.data_ptr()), C.c_void_p(offs.data_ptr()), None,
                                0, C.byref(total))
    assert rc == A.APR_OK
    cnt = counts.cpu().numpy()
    off = offs.cpu().numpy()
    assert off[0] == 0 and np.array_equal(off[1:], np.cumsum(cnt)) and total.value == cnt.sum()
    ids = ds["id"].cpu().numpy()
    own = np.empty(n, np.int64)
    own[ids] = cnt
    assert np.array_equal(g["nneigh"], own + 1)
    del ctx, ds, rho, om, counts, offs, hd
    torch.cuda.empty_cache()
    tg, od, _ = oracle_balls(st, p, 2, 32, seed=23, forces=False)
    for k in ("h", "rho", "omega"):
        assert _rel(g[k][tg], od[k]) < TOL["fp32"], k
