"""Helpers for GPU parity tests: run the library on a numpy state and map
results back to particle ids; run the oracle on whole sets or sampled balls."""
import numpy as np
import torch
from scipy.spatial import cKDTree

import oracle
import paper_2409_11470_amd as A
from _balls import dependency_ball, oracle_grads


def params_for(p, precision, tol=None, **kw):
    d = dict(precision=A.APR_FP32 if precision == "fp32" else A.APR_FP64,
             eos=int(p.get("eos", 0)), periodic=int(bool(p.get("periodic", False))),
             box_lo=p.get("lo", (0, 0, 0)), box_hi=p.get("hi", (1, 1, 1)), m0=float(p["m0"]),
             hfact=float(p.get("hfact", 1.2)), cs0=float(p.get("cs0", 1.0)),
             q_cs=float(p.get("q_cs", 0.25)), r_ref=float(p.get("r_ref", 1.0)),
             gamma=float(p.get("gamma", 5.0 / 3.0)), av_alpha=float(p.get("alpha", 1.0)),
             av_beta=float(p.get("beta", 2.0)), max_iter=60, kernel=int(p.get("kernel", 0)),
             tol_h=tol if tol is not None else (1e-6 if precision == "fp32" else 1e-12))
    d.update(kw)
    return A.make_params(**d)


def by_id(ids, values, n):
    out = np.empty((n,) + values.shape[1:], values.dtype)
    out[ids] = values
    return out


def gpu_density(st, p, precision, tol=None):
    """Returns per-id arrays h, rho, omega, nneigh, iters, and the context and state."""
    ctx = A.Context(params_for(p, precision, tol))
    ds = A.DeviceState.from_numpy(st)
    n = ds.n
    A.apr_build_cells(ctx, ds)
    dt = ctx.dtype
    rho = torch.zeros(n, dtype=dt, device="cuda")
    om = torch.zeros(n, dtype=dt, device="cuda")
    nn = torch.zeros(n, dtype=torch.int32, device="cuda")
    it = torch.zeros(n, dtype=torch.int32, device="cuda")
    A.apr_density(ctx, ds, rho, om, nn, it)
    fails = A.apr_sync_status(ctx, raise_noconverge=False)
    ids = ds["id"].cpu().numpy()
    n0 = st["x"].shape[0]
    res = dict(h=by_id(ids, ds["h"].cpu().numpy(), n0),
               rho=by_id(ids, rho.double().cpu().numpy(), n0),
               omega=by_id(ids, om.double().cpu().numpy(), n0),
               nneigh=by_id(ids, nn.cpu().numpy(), n0), iters=by_id(ids, it.cpu().numpy(), n0),
               failures=fails)
    return res, ctx, ds, (rho, om)


def gpu_forces(ctx, ds, rho, om):
    n = ds.n
    dt = ctx.dtype
    out = {k: torch.zeros(n, dtype=dt, device="cuda") for k in ("ax", "ay", "az", "dudt", "vsig")}
    A.apr_forces(ctx, ds, rho, om, out["ax"], out["ay"], out["az"], out["dudt"], out["vsig"])
    A.apr_sync_status(ctx)
    ids = ds["id"].cpu().numpy()
    return {k: by_id(ids, v.double().cpu().numpy(), n) for k, v in out.items()}


def oracle_density(st, p, tol=1e-12, targets=None, h_in=None):
    h0 = st["h"] if targets is None else st["h"][targets]
    if h_in is not None:
        h0 = h_in
    return oracle.density(st["x"], st["y"], st["z"], st["level"], h0, m0=p["m0"],
                          hfact=p.get("hfact", 1.2), tol=tol, max_iter=60,
                          periodic=p.get("periodic", False), lo=p.get("lo", (0, 0, 0)),
                          hi=p.get("hi", (1, 1, 1)), targets=targets,
                          kernel=int(p.get("kernel", 0)))


def oracle_forces(st, p, h, rho, omega, targets=None):
    return oracle.forces(st["x"], st["y"], st["z"], st["vx"], st["vy"], st["vz"], st["u"],
                         st["level"], h, rho, omega, m0=p["m0"], eos=int(p.get("eos", 0)),
                         cs0=p.get("cs0", 1.0), q_cs=p.get("q_cs", 0.25),
                         r_ref=p.get("r_ref", 1.0), gamma=p.get("gamma", 5.0 / 3.0),
                         alpha=p.get("alpha", 1.0), beta=p.get("beta", 2.0),
                         periodic=p.get("periodic", False), lo=p.get("lo", (0, 0, 0)),
                         hi=p.get("hi", (1, 1, 1)), targets=targets,
                         kernel=int(p.get("kernel", 0)))


def sample_balls(st, p, nballs, ntarget, seed, hscale):
    """Targets: the ntarget particles nearest to each of nballs random
    particles.  Shell: every particle within (ball radius + 4.5 hscale) of a
    ball centre, i.e. all particles that can be a target's neighbour or a
    neighbour's neighbour.  Returns (targets, shell) index arrays."""
    rng = np.random.default_rng(seed)
    n = st["x"].shape[0]
    pos = np.stack([st["x"], st["y"], st["z"]], 1)
    L = np.asarray(p.get("hi", (1, 1, 1)), float) - np.asarray(p.get("lo", (0, 0, 0)), float)
    per = bool(p.get("periodic", False))
    tg, sh = [], []
    for c in rng.choice(n, nballs, replace=False):
        d = pos - pos[c]
        if per:
            d -= L * np.round(d / L)
        r = np.sqrt((d * d).sum(1))
        order = np.argsort(r, kind="stable")[:ntarget]
        rb = r[order[-1]]
        tg.append(order)
        sh.append(np.nonzero(r < rb + 4.5 * hscale)[0])
    return np.unique(np.concatenate(tg)), np.unique(np.concatenate(sh))


def oracle_balls(st, p, nballs, ntarget, seed, tol=1e-12, forces=True, safety=1.5,
                 centres=None):
    """The FP64 oracle, exact on sampled targets of a large set: the ntarget
    particles nearest to each of nballs random particles (ball radius rb).
    Every particle b gets the reach bound R_b = 2 safety h0_b (h0 the initial
    h).  Solved set I: the b within rb + max(2 safety max h0(targets), R_b) of
    the ball centre, which holds every neighbour of a target under the
    symmetric criterion; sources: the union of the balls of radius R_b about
    the b in I (selected with a k-d tree; centres, if given, replace the random
    ball centres).  The
    density is solved for I over the sources and the forces summed on the
    targets over I.  Checked afterwards: every solved h <= safety h0, so each
    bound held for the solved particles.
    Returns (targets [global index], density dict, forces dict or None)."""
    rng = np.random.default_rng(seed)
    n = st["x"].shape[0]
    pos = np.stack([st["x"], st["y"], st["z"]], 1)
    reach = 2.0 * safety * st["h"]
    lo = np.asarray(p.get("lo", (0, 0, 0)), float)
    L = np.asarray(p.get("hi", (1, 1, 1)), float) - lo
    per = bool(p.get("periodic", False))
    T, I, S = [], [], []
    if centres is None:
        centres = rng.choice(n, nballs, replace=False)
    for c in centres:
        d = pos - pos[c]
        if per:
            d -= L * np.round(d / L)
        r = np.sqrt((d * d).sum(1))
        order = np.argsort(r, kind="stable")[:ntarget]
        rb = r[order[-1]]
        inner = r - rb < np.maximum(reach[order].max(), reach)
        rs = float(np.max(r[inner] + reach[inner]))
        cand = np.nonzero(r < rs)[0]
        box = L if per else None
        tree = cKDTree(pos[cand] - lo if per else pos[cand], boxsize=box)
        iin = np.nonzero(inner)[0]
        hits = tree.query_ball_point(pos[iin] - lo if per else pos[iin], reach[iin])
        T.append(order)
        I.append(iin)
        S.append(np.union1d(cand[np.unique(np.concatenate(hits))], iin))
    Tg = np.unique(np.concatenate(T))
    Sg = np.unique(np.concatenate(S))
    Ig = np.unique(np.concatenate(I))
    loc = np.full(n, -1, np.int64)
    loc[Sg] = np.arange(Sg.shape[0])
    sub = {k: st[k][Sg] for k in ("x", "y", "z", "vx", "vy", "vz", "u", "h", "level")}
    kw = dict(m0=p["m0"], hfact=p.get("hfact", 1.2), periodic=per, lo=tuple(lo),
              hi=tuple(lo + L), kernel=int(p.get("kernel", 0)))
    o = oracle.density(sub["x"], sub["y"], sub["z"], sub["level"], sub["h"][loc[Ig]], tol=tol,
                       max_iter=60, targets=loc[Ig], **kw)
    assert np.all(o["h"] <= safety * st["h"][Ig]), "a solved h exceeds its bound"
    ti = np.searchsorted(Ig, Tg)
    dens = {k: v[ti] for k, v in o.items() if isinstance(v, np.ndarray)}
    dens["failures"] = o["failures"]
    dens["sample"] = (Tg.size, Ig.size, Sg.size)
    if not forces:
        return Tg, dens, None
    m = Sg.shape[0]
    h, rho, om = np.full(m, 1e-12), np.ones(m), np.ones(m)
    h[loc[Ig]], rho[loc[Ig]], om[loc[Ig]] = o["h"], o["rho"], o["omega"]
    f = oracle.forces(sub["x"], sub["y"], sub["z"], sub["vx"], sub["vy"], sub["vz"], sub["u"],
                      sub["level"], h, rho, om, eos=int(p.get("eos", 0)),
                      cs0=p.get("cs0", 1.0), q_cs=p.get("q_cs", 0.25),
                      r_ref=p.get("r_ref", 1.0), gamma=p.get("gamma", 5.0 / 3.0),
                      alpha=p.get("alpha", 1.0), beta=p.get("beta", 2.0), targets=loc[Tg],
                      **{k: v for k, v in kw.items() if k != "hfact"})
    return Tg, dens, f


def gpu_grads(st, p, prec, cot, tol=None):
    """apr_sums (forward on the GPU, backward by apr_vjp) on the whole state
    with cotangents cot (as for oracle_grads); returns dL/dx [n, 3], dL/dm [n]
    in the order of st."""
    ctx = A.Context(params_for(p, prec, tol=tol))
    ds = A.DeviceState.from_numpy(st)
    x = ds["x"].clone().requires_grad_(True)
    y = ds["y"].clone().requires_grad_(True)
    z = ds["z"].clone().requires_grad_(True)
    m = (p["m0"] * torch.pow(2.0, -ds["level"].double())).requires_grad_(True)
    rho, h, ax, ay, az, du = A.apr_sums(ctx, ds, x, y, z, m)
    d = lambda a: torch.tensor(np.asarray(a), dtype=torch.float64, device="cuda")  # noqa: E731
    loss = ((d(cot["rho"]) * rho.double()).sum() + (d(cot["h"]) * h.double()).sum()
            + (d(cot["a"][:, 0]) * ax.double()).sum() + (d(cot["a"][:, 1]) * ay.double()).sum()
            + (d(cot["a"][:, 2]) * az.double()).sum() + (d(cot["du"]) * du.double()).sum())
    loss.backward()
    gx = torch.stack([x.grad, y.grad, z.grad], 1).cpu().numpy()
    gm = m.grad.cpu().numpy()
    del ctx, ds, x, y, z, m, rho, h, ax, ay, az, du, loss
    torch.cuda.empty_cache()
    return gx, gm


_BALL_CACHE = {}


def ball_vjp_check(key, st, p, prec, centre, ntarget=16, seed=0, gtol=None):
    """Sampled-ball parity of the adjoint on a large set: seeded N(0,1)
    cotangents on the rho, h, a and du/dt of the ntarget particles nearest to
    particle `centre` (scaled by the size of each quantity there, from the C
    oracle, so that no term hides the others) and zero elsewhere; the GPU's
    dL/dx and dL/dm over the whole set against torch autograd of the dense
    FP64 oracle solved on the dependency ball alone (dependency_ball).
    Gradients must vanish outside the ball and match inside it, relative to
    their max-norm, within gtol.  The oracle's side is cached per key (it does
    not depend on the form).  Returns the two relative errors."""
    n = st["x"].shape[0]
    if key not in _BALL_CACHE:
        T, S, solve, hS = dependency_ball(st, p, centre, ntarget)
        sub = {k: st[k][S] for k in ("x", "y", "z", "vx", "vy", "vz", "u", "level")}
        sub["h"] = hS
        ti = np.searchsorted(S, T)
        # sizes of the targets' rho, a, du/dt from the C oracle on the ball
        d = oracle.density(sub["x"], sub["y"], sub["z"], sub["level"], hS[ti], m0=p["m0"],
                           hfact=p.get("hfact", 1.2), tol=1e-14, max_iter=100,
                           periodic=bool(p.get("periodic", False)), lo=p.get("lo", (0, 0, 0)),
                           hi=p.get("hi", (1, 1, 1)), targets=ti, kernel=int(p.get("kernel", 0)))
        hh, rr, oo = hS.copy(), np.ones(S.size), np.ones(S.size)
        dn = oracle.density(sub["x"], sub["y"], sub["z"], sub["level"], hS[solve], m0=p["m0"],
                            hfact=p.get("hfact", 1.2), tol=1e-14, max_iter=100,
                            periodic=bool(p.get("periodic", False)),
                            lo=p.get("lo", (0, 0, 0)), hi=p.get("hi", (1, 1, 1)),
                            targets=np.nonzero(solve)[0], kernel=int(p.get("kernel", 0)))
        hh[solve], rr[solve], oo[solve] = dn["h"], dn["rho"], dn["omega"]
        f = oracle_forces(sub, p, hh, rr, oo, targets=ti)
        rng = np.random.default_rng(seed)
        cs = dict(rho=np.zeros(S.size), h=np.zeros(S.size), a=np.zeros((S.size, 3)),
                  du=np.zeros(S.size))
        amag = np.sqrt(f["ax"] ** 2 + f["ay"] ** 2 + f["az"] ** 2)
        cs["rho"][ti] = rng.normal(size=T.size) / d["rho"]
        cs["h"][ti] = rng.normal(size=T.size) / d["h"]
        cs["a"][ti] = rng.normal(size=(T.size, 3)) / np.maximum(amag, 1e-300)[:, None]
        # a target at rest among particles at rest has du/dt = 0 with no
        # dependence on x or m: no cotangent there
        du = np.abs(f["dudt"])
        cs["du"][ti] = np.where(du > 0, rng.normal(size=T.size) / np.where(du > 0, du, 1.0), 0.0)
        gx, gm = oracle_grads(sub, p, cs, solve=solve)
        cot = {k: np.zeros((n,) + v.shape[1:]) for k, v in cs.items()}
        for k in cot:
            cot[k][S] = cs[k]
        _BALL_CACHE[key] = (T, S, cot, gx, gm)
    T, S, cot, ox, om_ = _BALL_CACHE[key]
    gx, gm = gpu_grads(st, p, prec, cot)
    outside = np.ones(n, bool)
    outside[S] = False
    assert not np.any(gx[outside]) and not np.any(gm[outside]), "gradient outside the ball"
    ex = float(np.max(np.abs(gx[S] - ox)) / np.max(np.abs(ox)))
    em = float(np.max(np.abs(gm[S] - om_)) / np.max(np.abs(om_)))
    if gtol is not None:
        assert ex < gtol and em < gtol, (ex, em, T.size, S.size)
    return ex, em


def exact_counts(st, p, targets, h):
    """Neighbours of each target (self included) within 2 h[target] by the FP64
    predicate of the oracle: r^2 < (2h)^2 with r^2 = dx dx + dy dy + dz dz, no
    fused operations, dx = x_a - x_b at its minimum image in a periodic box.
    Candidates come from a k-d tree with a slightly larger radius; the
    predicate decides."""
    pos = np.stack([st["x"], st["y"], st["z"]], 1)
    per = bool(p.get("periodic", False))
    lo = np.asarray(p.get("lo", (0, 0, 0)), float)
    L = np.asarray(p.get("hi", (1, 1, 1)), float) - lo
    tree = cKDTree(pos - lo if per else pos, boxsize=L if per else None)
    out = np.empty(len(targets), np.int64)
    for k, a in enumerate(targets):
        R = 2.0 * float(h[a])
        cand = np.asarray(tree.query_ball_point((pos[a] - lo) if per else pos[a],
                                                R * (1.0 + 1e-9)), np.int64)
        d = pos[a] - pos[cand]
        if per:
            d = np.where(d > 0.5 * L, d - L, np.where(d < -0.5 * L, d + L, d))
        r2 = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2]
        out[k] = int(np.sum(r2 < R * R))
    return out
