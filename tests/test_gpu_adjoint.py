"""GPU adjoint (apr_vjp behind apr_sums) vs the gradient oracle and vs central
differences of the C oracle's forward.

Gradient parity: for seeded random cotangents of (rho, h, a, du/dt), the
position and mass gradients are compared with torch autograd of the dense
FP64 oracle forward; error = max |g_gpu - g_oracle| / max |g_oracle| per
gradient (x, y, z together; m), gates 1e-6 (FP64 form) and 1e-3 (FP32 form).
Difference checks: directional derivatives and the split-separation
derivative against central differences (eps 1e-6) of the C oracle at Newton
tolerance 1e-14, gates 1e-4 relative (FP64 form) and 1e-3 (FP32 form)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2409_11470_amd as A
import workloads as W
from _gpu import params_for
from oracle import adjoint as ADJ

pytestmark = pytest.mark.gpu

GTOL = {"fp64": 1e-6, "fp32": 1e-3}
FDTOL = {"fp64": 1e-4, "fp32": 1e-3}
G53 = 5.0 / 3.0


def _t(a, dev="cpu"):
    return torch.tensor(np.asarray(a), dtype=torch.float64, device=dev)


def _cluster(n, eos, seed_k, shift=0.0, vscale=0.4):
    st, dx = W.random_cluster(n, seed_k=seed_k, levels=(0, 1), vscale=vscale)
    st = dict(st, x=st["x"] + shift, y=st["y"] + shift)
    p = dict(m0=1.0, eos=eos, gamma=G53, cs0=1.0, q_cs=0.25, r_ref=1.0, alpha=1.0, beta=2.0,
             periodic=False, lo=(-1.0, -1.0, -1.0), hi=(3.0, 3.0, 3.0), hfact=1.2)
    return st, p


def _periodic_box(nside, seed_k=11):
    st, p = W.shock_box(nside=nside)
    n = st["x"].shape[0]
    rng = np.random.default_rng(seed_k)
    st = dict(st, vx=rng.normal(0, 0.3, n), vy=rng.normal(0, 0.3, n), vz=rng.normal(0, 0.3, n))
    return st, dict(p, m0=1.0 / n)


def _oracle_grads(st, p, cot):
    """autograd of the dense FP64 oracle: dL/dx [n, 3], dL/dm [n]."""
    x = _t(np.stack([st["x"], st["y"], st["z"]], 1)).requires_grad_(True)
    m = _t(p["m0"] * 2.0 ** -st["level"].astype(float)).requires_grad_(True)
    v = _t(np.stack([st["vx"], st["vy"], st["vz"]], 1))
    L = tuple(np.asarray(p["hi"], float) - np.asarray(p["lo"], float))
    rho, a, du, h, om = ADJ.forward(x, m, v, _t(st["u"]), _t(st["h"]), eos_kind=p["eos"],
                                    hfact=p["hfact"], cs0=p["cs0"], q_cs=p.get("q_cs", 0.25),
                                    r_ref=p.get("r_ref", 1.0), gamma=p["gamma"],
                                    alpha=p["alpha"], beta=p["beta"],
                                    periodic=p["periodic"], L=L,
                                    kernel=int(p.get("kernel", 0)))
    loss = ((_t(cot["rho"]) * rho).sum() + (_t(cot["h"]) * h).sum()
            + (_t(cot["a"]) * a).sum() + (_t(cot["du"]) * du).sum())
    gx, gm = torch.autograd.grad(loss, (x, m))
    return gx.numpy(), gm.numpy()


def _gpu_grads(st, p, prec, cot, tol=None):
    ctx = A.Context(params_for(p, prec, tol=tol))
    ds = A.DeviceState.from_numpy(st)
    x = ds["x"].clone().requires_grad_(True)
    y = ds["y"].clone().requires_grad_(True)
    z = ds["z"].clone().requires_grad_(True)
    m = (p["m0"] * torch.pow(2.0, -ds["level"].double())).requires_grad_(True)
    rho, h, ax, ay, az, du = A.apr_sums(ctx, ds, x, y, z, m)
    d = lambda a: _t(a, "cuda")  # noqa: E731
    loss = ((d(cot["rho"]) * rho.double()).sum() + (d(cot["h"]) * h.double()).sum()
            + (d(cot["a"][:, 0]) * ax.double()).sum() + (d(cot["a"][:, 1]) * ay.double()).sum()
            + (d(cot["a"][:, 2]) * az.double()).sum() + (d(cot["du"]) * du.double()).sum())
    loss.backward()
    gx = torch.stack([x.grad, y.grad, z.grad], 1).cpu().numpy()
    return gx, m.grad.cpu().numpy()


def _cotangents(n, seed, scale_h=1.0):
    rng = np.random.default_rng(seed)
    return dict(rho=rng.normal(size=n), h=scale_h * rng.normal(size=n),
                a=rng.normal(size=(n, 3)), du=rng.normal(size=n))


def _rel(g, o):
    return float(np.max(np.abs(g - o)) / np.max(np.abs(o)))


CASES = [
    ("adiabatic", lambda: _cluster(343, 2, 400)),
    ("isothermal", lambda: _cluster(343, 0, 401)),
    ("locally_isothermal", lambda: _cluster(343, 1, 402, shift=1.3)),
    ("periodic_mixed_mass", lambda: _periodic_box(12)),
]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_vjp_matches_oracle_gradient(name, make, prec):
    st, p = make()
    n = st["x"].shape[0]
    cot = _cotangents(n, 7)
    ox, om = _oracle_grads(st, p, cot)
    gx, gm = _gpu_grads(st, p, prec, cot)
    ex, em = _rel(gx, ox), _rel(gm, om)
    print(f"{name} {prec}: x {ex:.2e} m {em:.2e}")
    assert ex < GTOL[prec], ex
    assert em < GTOL[prec], em


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_vjp_many_cells(prec):
    # a jittered cluster spanning dozens of cells, two masses, moving
    st, p = _cluster(2744, 2, 403, vscale=0.6)
    cot = _cotangents(2744, 8)
    ox, om = _oracle_grads(st, p, cot)
    gx, gm = _gpu_grads(st, p, prec, cot)
    assert _rel(gx, ox) < GTOL[prec]
    assert _rel(gm, om) < GTOL[prec]


def test_density_only_cotangent():
    # only rho_bar: the force pass is skipped inside apr_vjp
    st, p = _cluster(343, 2, 404)
    n = st["x"].shape[0]
    rng = np.random.default_rng(9)
    cot = dict(rho=rng.normal(size=n), h=np.zeros(n), a=np.zeros((n, 3)), du=np.zeros(n))
    ox, om = _oracle_grads(st, p, cot)
    ctx = A.Context(params_for(p, "fp64"))
    ds = A.DeviceState.from_numpy(st)
    A.apr_build_cells(ctx, ds)
    rho = torch.empty(n, dtype=torch.float64, device="cuda")
    omg = torch.empty_like(rho)
    A.apr_density(ctx, ds, rho, omg)
    A.apr_sync_status(ctx)
    ids = ds["id"].cpu().numpy()
    rb = _t(cot["rho"][ids], "cuda")
    xb, yb, zb, mb = A.apr_vjp(ctx, ds, rho, omg, rho_bar=rb)
    g = np.empty((n, 3))
    g[ids] = torch.stack([xb, yb, zb], 1).cpu().numpy()
    gm = np.empty(n)
    gm[ids] = mb.cpu().numpy()
    assert _rel(g, ox) < 1e-6
    assert _rel(gm, om) < 1e-6


def test_zero_cotangent_gives_zero():
    st, p = _cluster(125, 2, 405)
    n = st["x"].shape[0]
    z = dict(rho=np.zeros(n), h=np.zeros(n), a=np.zeros((n, 3)), du=np.zeros(n))
    gx, gm = _gpu_grads(st, p, "fp64", z)
    assert np.all(gx == 0.0) and np.all(gm == 0.0)


def _c_loss(st, p, x, wr, wa, wu):
    d = oracle.density(x[:, 0], x[:, 1], x[:, 2], st["level"], st["h"], m0=p["m0"], tol=1e-14,
                       max_iter=100, lo=p["lo"], hi=p["hi"])
    assert d["failures"] == 0
    f = oracle.forces(x[:, 0], x[:, 1], x[:, 2], st["vx"], st["vy"], st["vz"], st["u"],
                      st["level"], d["h"], d["rho"], d["omega"], m0=p["m0"], eos=p["eos"],
                      gamma=p["gamma"], alpha=p["alpha"], beta=p["beta"], lo=p["lo"], hi=p["hi"])
    a = np.stack([f["ax"], f["ay"], f["az"]], 1)
    return np.sum(wr * d["rho"]) + np.sum(wa * a) + np.sum(wu * f["dudt"])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_vjp_matches_differences(prec):
    st, p = _cluster(216, 2, 406)
    n = st["x"].shape[0]
    cot = _cotangents(n, 10, scale_h=0.0)
    gx, _ = _gpu_grads(st, p, prec, cot)
    x0 = np.stack([st["x"], st["y"], st["z"]], 1)
    rng = np.random.default_rng(12)
    eps = 1e-6
    for k in range(8):
        dirn = rng.normal(size=(n, 3))
        fd = (_c_loss(st, p, x0 + eps * dirn, cot["rho"], cot["a"], cot["du"])
              - _c_loss(st, p, x0 - eps * dirn, cot["rho"], cot["a"], cot["du"])) / (2 * eps)
        an = float(np.sum(gx * dirn))
        scale = max(abs(fd), 1e-3 * float(np.sum(np.abs(gx * dirn))))
        assert abs(an - fd) < FDTOL[prec] * scale, (k, an, fd)


# ------------------------------------------------------------ split separation
def _split_setup():
    """Particles inside r < 0.3 of the cluster centre split once (tangential
    axis, r_sep = 0.2 h).  Returns the unsplit state, the split state, the
    pairs (+ child slot a, - child slot b), the parents' reference densities
    and the per-unit-separation offsets e = h_parent w."""
    st, p = _cluster(512, 2, 407, vscale=0.0)
    p = dict(p, r_sep_factor=0.2, nn_cap=0.0)
    zones = [dict(c=(0.5, 0.5, 0.5), r=(0.3,), ell=(1,))]
    d0 = oracle.density(st["x"], st["y"], st["z"], st["level"], st["h"], m0=1.0, tol=1e-14,
                        max_iter=100, lo=p["lo"], hi=p["hi"])
    st0 = dict(st, h=d0["h"], level=np.zeros_like(st["level"]))
    d0 = oracle.density(st0["x"], st0["y"], st0["z"], st0["level"], st0["h"], m0=1.0,
                        tol=1e-14, max_iter=100, lo=p["lo"], hi=p["hi"])
    st0["h"] = d0["h"]
    s1 = oracle.split_merge(st0, zones, step=1, seed=5, r_sep_factor=0.2, nn_cap=0.0,
                                  split_mode=0, background=0, derefine=False, periodic=False,
                                  lo=p["lo"], hi=p["hi"], dnn=None, cap=2 * 512, do_split=True,
                                  do_merge=False)
    n0 = st0["x"].shape[0]
    n1 = s1["x"].shape[0]
    split = np.nonzero(s1["level"][:n0] == 1)[0]
    assert n1 - n0 == split.size > 20
    pa, pb = split, n0 + np.arange(split.size)
    X1 = np.stack([s1["x"], s1["y"], s1["z"]], 1)
    e = (X1[pa] - X1[pb]) / (2 * 0.2)
    centre = 0.5 * (X1[pa] + X1[pb])
    rho_ref = d0["rho"][split]
    return s1, p, pa, pb, e, centre, rho_ref


def _rsep_positions(X1, pa, pb, centre, e, r):
    X = X1.copy()
    X[pa] = centre + r * e
    X[pb] = centre - r * e
    return X


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_split_separation_gradient(prec):
    s1, p, pa, pb, e, centre, rho_ref = _split_setup()
    n = s1["x"].shape[0]
    X1 = np.stack([s1["x"], s1["y"], s1["z"]], 1)

    def c_loss(r):
        X = _rsep_positions(X1, pa, pb, centre, e, r)
        d = oracle.density(X[:, 0], X[:, 1], X[:, 2], s1["level"], s1["h"], m0=1.0, tol=1e-14,
                           max_iter=100, lo=p["lo"], hi=p["hi"])
        assert d["failures"] == 0
        return float(np.sum((d["rho"][pa] - rho_ref) ** 2 + (d["rho"][pb] - rho_ref) ** 2))

    r0, eps = 0.2, 1e-6
    fd = (c_loss(r0 + eps) - c_loss(r0 - eps)) / (2 * eps)

    # GPU: positions as a differentiable function of r, density by apr_sums
    ctx = A.Context(params_for(p, prec))
    ds = A.DeviceState.from_numpy(dict(s1, vx=np.zeros(n), vy=np.zeros(n), vz=np.zeros(n)))
    r = torch.tensor(r0, dtype=torch.float64, device="cuda", requires_grad=True)
    base = _t(X1, "cuda")
    ea, eb = _t(e, "cuda"), _t(centre, "cuda")
    ia, ib = torch.as_tensor(pa, device="cuda"), torch.as_tensor(pb, device="cuda")
    Xa, Xb = eb + r * ea, eb - r * ea
    X = base.index_put((ia,), Xa).index_put((ib,), Xb)
    rho, *_ = A.apr_sums(ctx, ds, X[:, 0].contiguous(), X[:, 1].contiguous(),
                         X[:, 2].contiguous())
    ref = _t(rho_ref, "cuda")
    loss = ((rho.double()[ia] - ref) ** 2 + (rho.double()[ib] - ref) ** 2).sum()
    loss.backward()
    an = float(r.grad)
    print(f"r_sep gradient {prec}: {an:.10e} fd {fd:.10e}")
    assert abs(an - fd) < FDTOL[prec] * abs(fd), (an, fd)
