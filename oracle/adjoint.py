"""Gradient oracle for the density and force sums (test infrastructure only).

Dense PyTorch CPU float64: every pair of particles is formed explicitly and
masked by the kernel support, so this is only for a few thousand particles.
The forward follows the same definitions as apr_oracle.c (M4 or Wendland C2
kernel, h-rho
relation h = h_fact (m/rho)^(1/3), grad-h Omega, per-particle artificial
viscosity, isothermal / locally isothermal / adiabatic EOS); the gradient is
torch autograd of it.

The smoothing length is implicit.  h* is first converged by Newton without
gradients; then one Newton step is taken from h* with F'(h*) held constant,
    h = h* - F(h*; x, m) / F'(h*),
whose value equals h* to the solver tolerance and whose derivative is the
implicit-function-theorem one, dh/dp = -(dF/dp) / F'.

A subset of a large set can be solved alone: with ``solve`` (a bool mask),
only those particles' h solve the h-rho relation; the others keep the given
h0 as a constant (their own neighbourhoods may be incomplete in the subset,
and a loss that depends on their h only through which pairs exist is exact
when h0 is their converged value).
"""
import math

import torch

PI = math.pi


def _m4(q):
    """f, f', f'' of the M4 spline (zero for q >= 2)."""
    t = 2.0 - q
    inner = q < 1.0
    outer = (q >= 1.0) & (q < 2.0)
    f = torch.where(inner, 1.0 - 1.5 * q * q + 0.75 * q ** 3,
                    torch.where(outer, 0.25 * t ** 3, torch.zeros_like(q)))
    df = torch.where(inner, -3.0 * q + 2.25 * q * q,
                     torch.where(outer, -0.75 * t * t, torch.zeros_like(q)))
    return f, df


def _wc2(q):
    """f, f' of the Wendland C2 kernel, 21/16 (1 - q/2)^4 (1 + 2q) (zero for q >= 2)."""
    u = torch.clamp(1.0 - 0.5 * q, min=0.0)
    f = (21.0 / 16.0) * u ** 4 * (1.0 + 2.0 * q)
    df = -(105.0 / 16.0) * q * u ** 3
    return f, df


def _kern(q, kernel):
    return _wc2(q) if kernel == 1 else _m4(q)


def _pairs(x, periodic, L):
    d = x[:, None, :] - x[None, :, :]
    if periodic:
        Lt = torch.as_tensor(L, dtype=x.dtype)
        d = d - Lt * torch.round(d / Lt)
    n = x.shape[0]
    eye = torch.eye(n, dtype=torch.bool)
    r2 = (d * d).sum(-1)
    # r = 0 only on the diagonal here; keep its gradient finite
    r = torch.sqrt(torch.where(eye, torch.ones_like(r2), r2))
    r = torch.where(eye, torch.zeros_like(r), r)
    return d, r, eye


def _rho_terms(r, h, m, kernel=0):
    """rho_sum(h) and sum_b m_b dW/dh for every a (h is per row a)."""
    q = r / h[:, None]
    f, df = _kern(q, kernel)
    hh = h[:, None]
    W = f / (PI * hh ** 3)
    dWdh = -(3.0 * f + q * df) / (PI * hh ** 4)
    return (m[None, :] * W).sum(1), (m[None, :] * dWdh).sum(1)


def converge_h(x, m, h0, hfact=1.2, tol=1e-14, max_iter=100, periodic=False, L=(1, 1, 1),
               kernel=0, solve=None):
    with torch.no_grad():
        _, r, _ = _pairs(x, periodic, L)
        h = h0.clone()
        for _ in range(max_iter):
            rs, drs = _rho_terms(r, h, m, kernel)
            rhoh = m * (hfact / h) ** 3
            F = rs - rhoh
            dF = drs + 3.0 * rhoh / h
            hn = torch.where(dF > 0, h - F / dF, hfact * (m / rs) ** (1.0 / 3.0))
            hn = torch.minimum(torch.maximum(hn, 0.5 * h), 2.0 * h)
            done = (hn - h).abs() < tol * h
            if solve is not None:
                done = done | ~solve
            h = torch.where(done, h, hn)
            if bool(done.all()):
                break
        return h


def eos(x, rho, u, eos, cs0=1.0, q_cs=0.25, r_ref=1.0, gamma=5.0 / 3.0):
    if eos == 0:
        c = torch.full_like(rho, cs0)
        return cs0 * cs0 * rho, c
    if eos == 1:
        R = torch.sqrt(x[:, 0] ** 2 + x[:, 1] ** 2)
        c = cs0 * (R / r_ref) ** (-q_cs)
        return c * c * rho, c
    P = (gamma - 1.0) * rho * u
    return P, torch.sqrt(gamma * P / rho)


def forward(x, m, v, u, h0, *, eos_kind, hfact=1.2, cs0=1.0, q_cs=0.25, r_ref=1.0,
            gamma=5.0 / 3.0, alpha=1.0, beta=2.0, periodic=False, L=(1, 1, 1), kernel=0,
            solve=None):
    """rho [n], a [n, 3], du/dt [n], h [n], Omega [n] as differentiable functions
    of x [n, 3] and m [n] (v, u held fixed).  kernel: 0 M4, 1 Wendland C2.
    solve (optional bool [n]): only those h solve the h-rho relation; the
    others stay at h0, constants."""
    hs = converge_h(x.detach(), m.detach(), h0, hfact=hfact, periodic=periodic, L=L,
                    kernel=kernel, solve=solve)
    d, r, eye = _pairs(x, periodic, L)
    # implicit h: one Newton step from h* with F'(h*) held fixed
    rs, drs = _rho_terms(r, hs, m, kernel)
    rhoh = m * (hfact / hs) ** 3
    F = rs - rhoh
    dF = (drs + 3.0 * rhoh / hs).detach()
    h = hs - F / dF
    if solve is not None:
        h = torch.where(solve, h, h0)
    rho, drho = _rho_terms(r, h, m, kernel)
    omega = 1.0 + h * drho / (3.0 * rho)
    P, c = eos(x, rho, u, eos_kind, cs0, q_cs, r_ref, gamma)
    # pair terms, b != a, r < 2 max(h_a, h_b)
    ha, hb = h[:, None], h[None, :]
    qa, qb = r / ha, r / hb
    _, dfa = _kern(qa, kernel)
    _, dfb = _kern(qb, kernel)
    Fa = dfa / (PI * ha ** 4)
    Fb = dfb / (PI * hb ** 4)
    rsafe = torch.where(eye, torch.ones_like(r), r)
    rhat = d / rsafe[..., None]
    dv = v[:, None, :] - v[None, :, :]
    vdr = (dv * rhat).sum(-1)
    appr = vdr < 0
    vsa = alpha * c[:, None] + beta * vdr.abs()
    vsb = alpha * c[None, :] + beta * vdr.abs()
    qA = torch.where(appr, -0.5 * rho[:, None] * vsa * vdr, torch.zeros_like(vdr))
    qB = torch.where(appr, -0.5 * rho[None, :] * vsb * vdr, torch.zeros_like(vdr))
    Aa = (P[:, None] + qA) / (omega[:, None] * rho[:, None] ** 2)
    Bb = (P[None, :] + qB) / (omega[None, :] * rho[None, :] ** 2)
    pair = (~eye) & ((r < 2.0 * ha) | (r < 2.0 * hb))
    term = torch.where(pair, m[None, :] * (Aa * Fa + Bb * Fb), torch.zeros_like(r))
    a = -(term[..., None] * rhat).sum(1)
    du = torch.where(pair, m[None, :] * Aa * vdr * Fa, torch.zeros_like(r)).sum(1)
    return rho, a, du, h, omega
