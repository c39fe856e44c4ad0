"""Sampled-ball helpers of the gradient checks that touch only the oracle
(no GPU code): the dependency set of a loss on a few targets, and the dense
gradient oracle on such a set."""
import numpy as np
import torch
from scipy.spatial import cKDTree

import oracle


def dependency_ball(st, p, centre, ntarget, safety=1.5):
    """Index sets for a sampled-ball gradient check, from the C oracle's own
    converged h: T, the ntarget particles nearest to particle `centre`; N1,
    every particle that pairs with a target (r < 2 max(h_t, h_b)); N2, every
    particle within 2 h_b of one in N1 (the sources of N1's densities).  A
    loss on the targets' rho, h, a and du/dt depends on the positions and
    masses of S = T + N1 + N2 and, through the pair criterion, on the h of
    N2; solved alone, S gives its exact gradient when T + N1 solve the h-rho
    relation (their neighbourhoods lie in S) and N2 keeps the converged h.
    The searches use the bound h <= safety h0 (h0 the state's h, checked on
    every solved h), so the supersets they find hold N1, N2 and the sources
    of their densities.  Returns (T, S, solve mask over S, h over S)."""
    n = st["x"].shape[0]
    pos = np.stack([st["x"], st["y"], st["z"]], 1)
    lo = np.asarray(p.get("lo", (0, 0, 0)), float)
    L = np.asarray(p.get("hi", (1, 1, 1)), float) - lo
    per = bool(p.get("periodic", False))
    tree = cKDTree(pos - lo if per else pos, boxsize=L if per else None)
    q = (lambda P: P - lo) if per else (lambda P: P)
    R = 2.0 * safety * st["h"]   # support bound of every particle

    def near(I, radius):
        hits = tree.query_ball_point(q(pos[I]), radius)
        return np.unique(np.concatenate([np.asarray(x, np.int64) for x in hits] + [I]))

    def sep2(A, B):
        d = pos[A][:, None, :] - pos[B][None, :, :]
        if per:
            d -= L * np.round(d / L)
        return (d * d).sum(-1)
    _, T = tree.query(q(pos[centre:centre + 1]), ntarget)
    T = np.sort(np.asarray(T, np.int64).reshape(-1))
    # superset of N1: within R_t of a target, or within R_b of it (b near)
    c1 = near(T, 3.0 * R[T].max())
    J1 = c1[(np.sqrt(sep2(c1, T)) < np.maximum(R[c1][:, None], R[T][None, :])).any(1)]
    J2 = near(J1, R[J1])               # superset of N2
    src = near(J2, R[J2])              # every source of J2's densities
    loc = np.full(n, -1, np.int64)
    loc[src] = np.arange(src.size)
    o = oracle.density(st["x"][src], st["y"][src], st["z"][src], st["level"][src], st["h"][J2],
                       m0=p["m0"], hfact=p.get("hfact", 1.2), tol=1e-14, max_iter=100,
                       periodic=per, lo=tuple(lo), hi=tuple(lo + L), targets=loc[J2],
                       kernel=int(p.get("kernel", 0)))
    assert o["failures"] == 0 and np.all(o["h"] <= safety * st["h"][J2]), "bound violated"
    hc = np.full(n, np.nan)
    hc[J2] = o["h"]
    N1 = np.union1d(T, J1[(sep2(J1, T) < (2.0 * np.maximum(hc[J1][:, None],
                                                          hc[T][None, :])) ** 2).any(1)])
    hits = tree.query_ball_point(q(pos[N1]), 2.0 * hc[N1])
    N2 = np.unique(np.concatenate([np.asarray(x, np.int64) for x in hits]))
    S = np.union1d(N1, N2)
    assert np.all(np.isin(S, J2))
    return T, S, np.isin(S, N1), hc[S]


def oracle_grads(st, p, cot, solve=None):
    """Torch autograd of the dense FP64 gradient oracle on the whole of st:
    dL/dx [n, 3], dL/dm [n] for L = sum rho_bar rho + h_bar h + a_bar . a +
    dudt_bar du/dt (cot holds rho, h, a [n, 3], du); solve (optional): only
    those h solve the h-rho relation, the others keep st["h"]."""
    from oracle import adjoint as ADJ
    t = lambda a: torch.tensor(np.asarray(a), dtype=torch.float64)  # noqa: E731
    x = t(np.stack([st["x"], st["y"], st["z"]], 1)).requires_grad_(True)
    m = t(p["m0"] * 2.0 ** -st["level"].astype(float)).requires_grad_(True)
    v = t(np.stack([st["vx"], st["vy"], st["vz"]], 1))
    L = tuple(np.asarray(p.get("hi", (1, 1, 1)), float) - np.asarray(p.get("lo", (0, 0, 0)), float))
    rho, a, du, h, om = ADJ.forward(x, m, v, t(st["u"]), t(st["h"]), eos_kind=int(p["eos"]),
                                    hfact=p.get("hfact", 1.2), cs0=p.get("cs0", 1.0),
                                    q_cs=p.get("q_cs", 0.25), r_ref=p.get("r_ref", 1.0),
                                    gamma=p.get("gamma", 5.0 / 3.0), alpha=p.get("alpha", 1.0),
                                    beta=p.get("beta", 2.0),
                                    periodic=bool(p.get("periodic", False)), L=L,
                                    kernel=int(p.get("kernel", 0)),
                                    solve=None if solve is None else torch.as_tensor(solve))
    loss = ((t(cot["rho"]) * rho).sum() + (t(cot["h"]) * h).sum()
            + (t(cot["a"]) * a).sum() + (t(cot["du"]) * du).sum())
    gx, gm = torch.autograd.grad(loss, (x, m))
    return gx.numpy(), gm.numpy()
