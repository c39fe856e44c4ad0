"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws particle sets: positions, velocities, thermal energy,
refinement levels, ids and an initial smoothing-length guess.  It holds none of
the method's arithmetic (no kernel sums, no h-rho solve, no forces, no
split/merge) and is shared, as plain numpy arrays, by the CPU oracle and the
GPU library's tests and benchmark.

The paper's own initial conditions (the HD 142527 set-up, the planet-disc and
flyby runs) are not available; every workload here is a synthetic stand-in with
the same shape: a periodic lattice box, a Keplerian disc around one point mass
with a refinement sphere, and a circumbinary disc with two nested refinement
levels.  Seeds are numpy PCG64 with seed 2409114700 + workload number.

A state is a dict of numpy arrays
    x, y, z, vx, vy, vz, u, h : float64 [n]
    level : int8 [n]          refinement level (mass m0 / 2**level)
    id    : int64 [n]         persistent particle id
and the scalar next_id, plus a dict `params` with the physical set-up.
"""
import numpy as np

SEED_BASE = 2409114700


def _rng(k):
    return np.random.Generator(np.random.PCG64(SEED_BASE + k))


def _state(x, y, z, vx, vy, vz, u, h, level):
    n = x.shape[0]
    return dict(x=np.ascontiguousarray(x, np.float64), y=np.ascontiguousarray(y, np.float64),
                z=np.ascontiguousarray(z, np.float64), vx=np.ascontiguousarray(vx, np.float64),
                vy=np.ascontiguousarray(vy, np.float64), vz=np.ascontiguousarray(vz, np.float64),
                u=np.ascontiguousarray(u, np.float64), h=np.ascontiguousarray(h, np.float64),
                level=np.ascontiguousarray(level, np.int8), id=np.arange(n, dtype=np.int64),
                next_id=n)


def lattice_positions(nside, L=1.0):
    """Simple cubic lattice ((i + 1/2) L/nside, ...), x fastest."""
    g = (np.arange(nside) + 0.5) * (L / nside)
    zz, yy, xx = np.meshgrid(g, g, g, indexing="ij")
    return xx.ravel().copy(), yy.ravel().copy(), zz.ravel().copy()


def lattice_box(nside=16, seed_k=1, vjitter=1e-3):
    """Workload 1: 16^3 equal-mass lattice in the periodic unit box, rho = 1,
    isothermal cs = 1, velocity jitter U(-1e-3, 1e-3) per component."""
    rng = _rng(seed_k)
    x, y, z = lattice_positions(nside)
    n = x.shape[0]
    v = rng.uniform(-vjitter, vjitter, size=(3, n))
    dx = 1.0 / nside
    st = _state(x, y, z, v[0], v[1], v[2], np.zeros(n), np.full(n, 1.2 * dx),
                np.zeros(n, np.int8))
    params = dict(m0=1.0 / n, periodic=True, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), eos=0,
                  cs0=1.0, gamma=5.0 / 3.0, alpha=1.0, beta=2.0, hfact=1.2)
    return st, params


def shock_box(nside=64, seed_k=2, jitter=0.1):
    """Workload 2: 64^3 lattice in the periodic unit box with U(-0.1, 0.1) dx
    jitter per axis.  x < 0.5: rho = 1, P = 1; x >= 0.5: rho = 0.125, P = 0.1.
    One lattice for both sides, so the density contrast of 8 is carried by the
    masses: level 0 (m0 = 2^-18) on the left, level 3 (m0/8) on the right.
    Adiabatic gamma = 5/3, u = P/((gamma-1) rho), v = 0."""
    rng = _rng(seed_k)
    x, y, z = lattice_positions(nside)
    n = x.shape[0]
    dx = 1.0 / nside
    j = rng.uniform(-jitter * dx, jitter * dx, size=(3, n))
    x, y, z = x + j[0], y + j[1], z + j[2]
    left = x < 0.5
    gamma = 5.0 / 3.0
    u = np.where(left, 1.0 / ((gamma - 1.0) * 1.0), 0.1 / ((gamma - 1.0) * 0.125))
    level = np.where(left, 0, 3).astype(np.int8)
    z0 = np.zeros(n)
    st = _state(x, y, z, z0, z0, z0, u, np.full(n, 1.2 * dx), level)
    params = dict(m0=2.0 ** -18, periodic=True, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), eos=2,
                  cs0=1.0, gamma=gamma, alpha=1.0, beta=2.0, hfact=1.2)
    return st, params


def _disc_samples(rng, n, r_in, r_out, M_star, cs_in, q_cs, zone=None):
    """Monte-Carlo Keplerian disc: Sigma ~ R^-1 (uniform in R), uniform phi,
    Gaussian z with H = cs(R)/Omega_K(R), cs = cs_in (R/r_in)^-q, Keplerian
    azimuthal velocity about a central mass M_star at the origin (G = 1)."""
    R = rng.uniform(r_in, r_out, n)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    cs = cs_in * (R / r_in) ** (-q_cs)
    om = np.sqrt(M_star / R ** 3)
    H = cs / om
    z = rng.normal(0.0, 1.0, n) * H
    x, y = R * np.cos(phi), R * np.sin(phi)
    vk = np.sqrt(M_star / R)
    vx, vy = -vk * np.sin(phi), vk * np.cos(phi)
    return x, y, z, vx, vy, np.zeros(n), R, H


def _disc_h_guess(R, z, H, m, M_disc, r_in, r_out):
    """1.2 times the mean interparticle spacing of the analytic number density
    (Sigma(R) = M_disc / (2 pi (r_out - r_in) R), Gaussian in z), floored so
    that very sparse particles start from a finite guess."""
    sig = M_disc / (2.0 * np.pi * (r_out - r_in) * R)
    rho = sig / (np.sqrt(2.0 * np.pi) * H) * np.exp(-0.5 * (z / H) ** 2)
    rho = np.maximum(rho, 1e-3 * sig / (np.sqrt(2.0 * np.pi) * H))
    return 1.2 * (m / rho) ** (1.0 / 3.0)


def planet_disc(n=1_000_000, seed_k=3):
    """Workload 3: 3D Keplerian disc about a unit point mass, R in [1, 10],
    Sigma ~ R^-1, H/R = 0.05 at R = 1, locally isothermal cs ~ R^-0.25,
    M_disc = 0.05; one refinement sphere r = 1 at (5, 0, 0), level 1; splits
    put children at +-0.5 h along seeded random axes."""
    rng = _rng(seed_k)
    r_in, r_out, M_disc = 1.0, 10.0, 0.05
    cs_in, q = 0.05, 0.25
    x, y, z, vx, vy, vz, R, H = _disc_samples(rng, n, r_in, r_out, 1.0, cs_in, q)
    m0 = M_disc / n
    h = _disc_h_guess(R, z, H, m0, M_disc, r_in, r_out)
    st = _state(x, y, z, vx, vy, vz, np.zeros(n), h, np.zeros(n, np.int8))
    zmax = float(np.max(np.abs(z))) * 1.5 + 1.0
    params = dict(m0=m0, periodic=False, lo=(-11.0, -11.0, -zmax), hi=(11.0, 11.0, zmax),
                  eos=1, cs0=cs_in, q_cs=q, r_ref=r_in, gamma=5.0 / 3.0, alpha=1.0, beta=2.0,
                  hfact=1.2, r_sep_factor=0.5, nn_cap=0.0, split_mode=1,
                  zones=[dict(c=(5.0, 0.0, 0.0), r=(1.0,), ell=(1,))],
                  sinks=[dict(x=(0.0, 0.0, 0.0), m=1.0, eps=0.0)], G=1.0)
    return st, params


def refine_box(nside=64, seed_k=4):
    """Workload 4: workload 2's particles plus a refinement sphere r = 0.45 at
    the box centre whose level (4) is above every particle's, so one pass
    splits every particle inside it by one level (about 1e5 parents into 2e5
    children).  Tangential split, r_sep = 0.2 h, no nearest-neighbour cap."""
    st, params = shock_box(nside=nside, seed_k=2)
    params = dict(params)
    params.update(zones=[dict(c=(0.5, 0.5, 0.5), r=(0.45,), ell=(4,))], r_sep_factor=0.2,
                  nn_cap=0.0, split_mode=0)
    return st, params


def hcp_positions(nx, ny, nz, a):
    """Hexagonal close-packed lattice of spacing a: nx per row along x, ny rows
    (spacing a sqrt(3)/2, odd rows shifted a/2), nz layers (spacing
    a sqrt(2/3), odd layers shifted by (a/2, a sqrt(3)/6)); ny and nz even, so
    the box (nx a, ny a sqrt(3)/2, nz a sqrt(2/3)) tiles periodically."""
    dy, dz = a * np.sqrt(3.0) / 2.0, a * np.sqrt(2.0 / 3.0)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    x = (i + 0.25 + 0.5 * (j % 2) + 0.5 * (k % 2)) * a
    y = (j + 0.25 + (k % 2) / 3.0) * dy
    z = (k + 0.5) * dz
    L = np.array([nx * a, ny * dy, nz * dz])
    return np.mod(x.ravel(), L[0]), y.ravel().copy(), z.ravel().copy(), L


def wave_box(nx=64, nz=12, seed_k=6, amp=0.02, noise=1e-4, vx=1e-3, hfact=1.2):
    """Workload 6, the sound-wave box of the paper's appendix A: a thin
    periodic box of width 1 in x and about 1 in y, hcp lattice with nx
    particles across (64 x 74 x 12 = 56832 at nx = 64), stretched along x so
    that rho = 1 + amp sin(2 pi x); adiabatic gamma = 5/3 with unperturbed
    sound speed 1, u perturbed with the same amplitude scaled by P0/rho0;
    v = (vx, 0, 0); x and y moved by U(-noise, noise).  Refinement: one
    cylinder along z of radius 0.1 about (0.5, 0.5) at level 1, tangential
    split at r_sep = 0.2 h with the nearest-neighbour cap 0.35.  nz (even) is
    the number of layers: 12 in the paper; the box stays at least 8 h thick, as
    periodic supports need, for any nx."""
    rng = _rng(seed_k)
    a = 1.0 / nx
    ny = 2 * int(round(nx / np.sqrt(3.0)))
    x0, y, z, L = hcp_positions(nx, ny, nz, a)
    L[0] = 1.0
    # stretch: the mass left of x is x + amp/(2 pi) (1 - cos 2 pi x) = x0
    x = x0.copy()
    for _ in range(50):
        g = x + amp / (2 * np.pi) * (1.0 - np.cos(2 * np.pi * x)) - x0
        x -= g / (1.0 + amp * np.sin(2 * np.pi * x))
    n = x.shape[0]
    x = np.mod(x + rng.uniform(-noise, noise, n), 1.0)
    y = np.mod(y + rng.uniform(-noise, noise, n) * L[1], L[1])
    gamma, cs0, rho0 = 5.0 / 3.0, 1.0, 1.0
    P0 = rho0 * cs0 * cs0 / gamma
    rho = rho0 + amp * np.sin(2 * np.pi * x)
    u = P0 / ((gamma - 1.0) * rho0) + amp * (P0 / rho0) * np.sin(2 * np.pi * x)
    m = rho0 * L[0] * L[1] * L[2] / n
    h = hfact * (m / rho) ** (1.0 / 3.0)
    st = _state(x, y, z, np.full(n, vx), np.zeros(n), np.zeros(n), u, h, np.zeros(n, np.int8))
    params = dict(m0=m, periodic=True, lo=(0.0, 0.0, 0.0), hi=tuple(float(v) for v in L),
                  eos=2, gamma=gamma, cs0=cs0, alpha=1.0, beta=2.0, hfact=hfact,
                  zones=[dict(c=(0.5, 0.5, 0.5 * L[2]), r=(0.1,), ell=(1,), shape=1)],
                  r_sep_factor=0.2, nn_cap=0.35, split_mode=0, amp=amp)
    return st, params


def circumbinary_disc(n0=6_550_000, seed_k=5):
    """Workload 5: circumbinary disc about two unit masses at separation 1 on
    a circular orbit (Omega_b = sqrt 2), R in [2, 20], Sigma ~ R^-1, H/R = 0.05
    at R = 2, cs ~ R^-0.25.  Two nested refinement levels centred on the
    binary's centre of mass: level 2 for r < 3, level 1 for 3 <= r < 4.  The
    refined regions are sampled directly at 2x and 4x the base number
    density with masses m0/2 and m0/4 (a multi-mass set-up), so the disc's
    mass density is continuous across the zone edges."""
    rng = _rng(seed_k)
    r_in, r_out, M_disc, Mtot = 2.0, 20.0, 0.05, 2.0
    cs_in, q = 0.05, 0.25
    m0 = M_disc / n0
    parts = []
    for k, lmin in enumerate((0, 1, 2, 2)):
        x, y, z, vx, vy, vz, R, H = _disc_samples(rng, n0, r_in, r_out, Mtot, cs_in, q)
        rs = np.sqrt(x * x + y * y + z * z)
        lev = np.where(rs < 3.0, 2, np.where(rs < 4.0, 1, 0))
        keep = lev >= lmin
        parts.append((x[keep], y[keep], z[keep], vx[keep], vy[keep], vz[keep], R[keep],
                      H[keep], lev[keep]))
    cat = [np.concatenate([p[i] for p in parts]) for i in range(9)]
    x, y, z, vx, vy, vz, R, H, lev = cat
    m = m0 / 2.0 ** lev
    # local number density is 2**lev times the base one, mass m0/2**lev
    h = _disc_h_guess(R, z, H, m0, M_disc, r_in, r_out) / 2.0 ** (lev / 3.0)
    st = _state(x, y, z, vx, vy, vz, np.zeros(x.shape[0]), h, lev.astype(np.int8))
    del m
    zmax = float(np.max(np.abs(z))) * 1.5 + 1.0
    params = dict(m0=m0, periodic=False, lo=(-21.0, -21.0, -zmax), hi=(21.0, 21.0, zmax),
                  eos=1, cs0=cs_in, q_cs=q, r_ref=r_in, gamma=5.0 / 3.0, alpha=1.0, beta=2.0,
                  hfact=1.2, r_sep_factor=0.2, nn_cap=0.35, split_mode=0,
                  zones=[dict(c=(0.0, 0.0, 0.0), r=(4.0, 3.0), ell=(1, 2))],
                  sinks=[dict(x=(0.5, 0.0, 0.0), m=1.0, eps=0.0),
                         dict(x=(-0.5, 0.0, 0.0), m=1.0, eps=0.0)],
                  G=1.0, omega_b=float(np.sqrt(2.0)))
    return st, params


def binary_positions(t, omega_b=np.sqrt(2.0), a=1.0):
    """Prescribed circular orbit of the two equal sinks at time t."""
    c, s = np.cos(omega_b * t), np.sin(omega_b * t)
    return np.array([[0.5 * a * c, 0.5 * a * s, 0.0], [-0.5 * a * c, -0.5 * a * s, 0.0]])


def random_cluster(n, seed_k=100, levels=(0,), spread=1.0, vscale=0.0):
    """Small non-periodic jittered-lattice cluster for pins and parity tests:
    particles on a cubic lattice of spacing 1/round(n^(1/3)) inside [0, spread)^3
    with 0.2-spacing jitter, levels drawn from `levels`, optional random
    velocities U(-vscale, vscale)."""
    rng = _rng(seed_k)
    side = max(2, int(round(n ** (1.0 / 3.0))))
    x, y, z = lattice_positions(side, L=spread)
    x, y, z = x[:n], y[:n], z[:n]
    m = x.shape[0]
    dx = spread / side
    j = rng.uniform(-0.2 * dx, 0.2 * dx, size=(3, m))
    lev = rng.choice(np.asarray(levels, dtype=np.int8), size=m)
    v = rng.uniform(-vscale, vscale, size=(3, m)) if vscale > 0 else np.zeros((3, m))
    u = rng.uniform(1.0, 2.0, size=m)
    st = _state(x + j[0], y + j[1], z + j[2], v[0], v[1], v[2], u, np.full(m, 1.2 * dx), lev)
    return st, dx
