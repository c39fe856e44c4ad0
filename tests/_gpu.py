"""Helpers for GPU parity tests: run the library on a numpy state and map
results back to particle ids; run the oracle on whole sets or sampled balls."""
import numpy as np
import torch
from scipy.spatial import cKDTree

import oracle
import paper_2409_11470_amd as A


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
