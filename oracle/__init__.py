"""Plain FP64 CPU oracle for the APR-SPH hot path (Nealon & Price 2024).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product library never does.  It
shares no code with the GPU library.  Arrays are numpy; the arithmetic lives in
``apr_oracle.c`` (brute-force O(N^2) neighbour search, FP64, no FMA
contraction) and, for gradients, in ``adjoint.py`` (dense PyTorch CPU float64).

Most functions below marshal arguments to the C code only.  The exceptions
hold oracle arithmetic of their own, in plain Python over those C calls:
``relax`` (the shuffle loop of Sec. 2.4), ``courant_bin``, ``accel_bins`` and
``step_bins`` (the individual timesteps of Sec. 2.5), each with its passage.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_LIB = None

_d = C.POINTER(C.c_double)
_i8 = C.POINTER(C.c_int8)
_i32 = C.POINTER(C.c_int32)
_i64 = C.POINTER(C.c_int64)
_u8 = C.POINTER(C.c_uint8)


def lib():
    """Load liboracle.so, building it first if it is not there."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        L.orc_num_threads.restype = C.c_int32
        L.orc_num_threads.argtypes = []
        L.orc_m4_f.restype = C.c_double
        L.orc_m4_f.argtypes = [C.c_double]
        L.orc_m4_df.restype = C.c_double
        L.orc_m4_df.argtypes = [C.c_double]
        L.orc_m4_d2f.restype = C.c_double
        L.orc_m4_d2f.argtypes = [C.c_double]
        for nm in ("orc_wc2_f", "orc_wc2_df", "orc_wc2_d2f"):
            getattr(L, nm).restype = C.c_double
            getattr(L, nm).argtypes = [C.c_double]
        for nm in ("orc_kf", "orc_kdf", "orc_kd2f"):
            getattr(L, nm).restype = C.c_double
            getattr(L, nm).argtypes = [C.c_int32, C.c_double]
        for nm in ("orc_wk", "orc_dwdhk"):
            getattr(L, nm).restype = C.c_double
            getattr(L, nm).argtypes = [C.c_int32, C.c_double, C.c_double]
        L.orc_w.restype = C.c_double
        L.orc_w.argtypes = [C.c_double, C.c_double]
        L.orc_dwdh.restype = C.c_double
        L.orc_dwdh.argtypes = [C.c_double, C.c_double]
        L.orc_density.restype = C.c_int64
        L.orc_density.argtypes = [C.c_int64, _d, _d, _d, _i8, C.c_double, C.c_double,
                                  C.c_double, C.c_int32, C.c_int32, _d, _d, C.c_int64, _i64,
                                  _d, _d, _d, _d, _i32, _d, _i32, C.c_int32]
        L.orc_neighbours.restype = None
        L.orc_neighbours.argtypes = [C.c_int64, _d, _d, _d, _d, C.c_int32, C.c_int32, _d, _d,
                                     C.c_int64, _i64, _i64, _i64, _i64]
        L.orc_eos.restype = None
        L.orc_eos.argtypes = [C.c_int64, C.c_int32, C.c_double, C.c_double, C.c_double,
                              C.c_double, _d, _d, _d, _d, _d, _d]
        L.orc_forces.restype = None
        L.orc_forces.argtypes = [C.c_int64, _d, _d, _d, _d, _d, _d, _d, _i8, _d, _d, _d,
                                 C.c_double, C.c_int32, C.c_double, C.c_double, C.c_double,
                                 C.c_double, C.c_double, C.c_double, C.c_int32, _d, _d,
                                 C.c_int64, _i64, _d, _d, _d, _d, _d, _d, _d, C.c_int32]
        L.orc_interp.restype = None
        L.orc_interp.argtypes = [C.c_int64, _d, _d, _d, C.c_int64, _d, _d, _d, _d, _d, _d, _d,
                                 C.c_int32, C.c_int32, _d, _d, _d, _d, _d]
        L.orc_kick.restype = None
        L.orc_kick.argtypes = [C.c_int64, _d, _d, _d, _d, _d, _d, _d, _d, C.c_double]
        L.orc_drift.restype = None
        L.orc_drift.argtypes = [C.c_int64, _d, _d, _d, _d, _d, _d, C.c_double, C.c_int32,
                                _d, _d]
        L.orc_sink_gravity.restype = None
        L.orc_sink_gravity.argtypes = [C.c_int64, _d, _d, _d, C.c_int32, _d, _d, _d,
                                       C.c_double, _d, _d, _d]
        L.orc_splitmix64.restype = C.c_uint64
        L.orc_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
        L.orc_zone_level.restype = C.c_int32
        L.orc_zone_level.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int32, _d, _i32,
                                     _d, _i32, _i32, C.c_int32, C.c_int32]
        L.orc_pair_tree.restype = C.c_int64
        L.orc_pair_tree.argtypes = [C.c_int64, _i64, _d, _d, _d, _i64, _d, _d, C.c_int64,
                                    _i64]
        L.orc_split_merge.restype = C.c_int32
        L.orc_split_merge.argtypes = [C.c_int64, C.c_int64, _d, _d, _d, _d, _d, _d, _d, _d,
                                      _i8, _i64, _i64, _d, C.c_int32, _d, _i32, _d, _i32,
                                      _i32, C.c_int32, C.c_int32, C.c_double, C.c_double,
                                      C.c_int32, C.c_uint64, C.c_int64, C.c_int32, _d, _d,
                                      C.c_int32, C.c_int32, _i64, _i64, _i64, _i64, _u8, _i64,
                                      _u8]
        _LIB = L
    return _LIB


def _p(a, t):
    if a is None:
        return None
    return a.ctypes.data_as(t)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _box(lo, hi):
    return _f64(np.asarray(lo, dtype=np.float64).reshape(3)), _f64(
        np.asarray(hi, dtype=np.float64).reshape(3))


def num_threads():
    return int(lib().orc_num_threads())


# --------------------------------------------------------------------- kernel
def m4_f(q):
    return lib().orc_m4_f(float(q))


def m4_df(q):
    return lib().orc_m4_df(float(q))


def m4_d2f(q):
    return lib().orc_m4_d2f(float(q))


KERNEL_M4, KERNEL_WC2 = 0, 1


def wc2_f(q):
    return lib().orc_wc2_f(float(q))


def wc2_df(q):
    return lib().orc_wc2_df(float(q))


def wc2_d2f(q):
    return lib().orc_wc2_d2f(float(q))


def kf(q, kernel=KERNEL_M4):
    """f(q) of the chosen kernel (W = f(q)/(pi h^3))."""
    return lib().orc_kf(int(kernel), float(q))


def kdf(q, kernel=KERNEL_M4):
    return lib().orc_kdf(int(kernel), float(q))


def kd2f(q, kernel=KERNEL_M4):
    return lib().orc_kd2f(int(kernel), float(q))


def w(r, h, kernel=KERNEL_M4):
    return lib().orc_wk(int(kernel), float(r), float(h))


def dwdh(r, h, kernel=KERNEL_M4):
    return lib().orc_dwdhk(int(kernel), float(r), float(h))


# -------------------------------------------------------------------- density
def density(x, y, z, level, h_in, *, m0, hfact=1.2, tol=1e-12, max_iter=50, periodic=False,
            lo=(0, 0, 0), hi=(1, 1, 1), targets=None, kernel=KERNEL_M4):
    """h-rho Newton solve for every target (all particles if targets is None).

    h_in is indexed like the targets.  Returns a dict of per-target arrays
    h, rho, omega, nneigh (self included), dnn, iters, and 'failures'."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    level = np.ascontiguousarray(level, dtype=np.int8)
    n = x.shape[0]
    tg = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    nt = n if tg is None else tg.shape[0]
    h_in = _f64(h_in)
    assert h_in.shape[0] == nt
    lo, hi = _box(lo, hi)
    out = dict(h=np.empty(nt), rho=np.empty(nt), omega=np.empty(nt),
               nneigh=np.empty(nt, np.int32), dnn=np.empty(nt), iters=np.empty(nt, np.int32))
    fails = lib().orc_density(n, _p(x, _d), _p(y, _d), _p(z, _d), _p(level, _i8), m0, hfact,
                              tol, max_iter, int(bool(periodic)), _p(lo, _d), _p(hi, _d), nt,
                              _p(tg, _i64), _p(h_in, _d), _p(out["h"], _d),
                              _p(out["rho"], _d), _p(out["omega"], _d),
                              _p(out["nneigh"], _i32), _p(out["dnn"], _d),
                              _p(out["iters"], _i32), int(kernel))
    out["failures"] = int(fails)
    return out


# ----------------------------------------------------------------- neighbours
def neighbours(x, y, z, h, *, symmetric=False, periodic=False, lo=(0, 0, 0), hi=(1, 1, 1),
               targets=None):
    """Brute-force neighbour lists (b != a) for a given h; returns a list of
    int64 arrays in ascending index order, one per target."""
    x, y, z, h = _f64(x), _f64(y), _f64(z), _f64(h)
    n = x.shape[0]
    tg = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    nt = n if tg is None else tg.shape[0]
    lo, hi = _box(lo, hi)
    counts = np.zeros(nt, np.int64)
    args = (n, _p(x, _d), _p(y, _d), _p(z, _d), _p(h, _d), int(bool(symmetric)),
            int(bool(periodic)), _p(lo, _d), _p(hi, _d), nt, _p(tg, _i64))
    lib().orc_neighbours(*args, _p(counts, _i64), None, None)
    offs = np.zeros(nt + 1, np.int64)
    np.cumsum(counts, out=offs[1:])
    lst = np.empty(max(int(offs[-1]), 1), np.int64)
    lib().orc_neighbours(*args, _p(counts, _i64), _p(offs, _i64), _p(lst, _i64))
    return [lst[offs[t]:offs[t + 1]].copy() for t in range(nt)]


# ------------------------------------------------------------------------ eos
EOS_ISOTHERMAL, EOS_LOCALLY_ISOTHERMAL, EOS_ADIABATIC = 0, 1, 2


def eos(x, y, rho, u=None, *, eos, cs0=1.0, q_cs=0.25, r_ref=1.0, gamma=5.0 / 3.0):
    x, y, rho = _f64(x), _f64(y), _f64(rho)
    u = None if u is None else _f64(u)
    n = x.shape[0]
    P, c = np.empty(n), np.empty(n)
    lib().orc_eos(n, eos, cs0, q_cs, r_ref, gamma, _p(x, _d), _p(y, _d), _p(rho, _d),
                  _p(u, _d), _p(P, _d), _p(c, _d))
    return P, c


# --------------------------------------------------------------------- forces
def forces(x, y, z, vx, vy, vz, u, level, h, rho, omega, *, m0, eos, cs0=1.0, q_cs=0.25,
           r_ref=1.0, gamma=5.0 / 3.0, alpha=1.0, beta=2.0, periodic=False, lo=(0, 0, 0),
           hi=(1, 1, 1), targets=None, kernel=KERNEL_M4):
    """Hydro acceleration, du/dt, vsig and the L1 bounds anorm, unorm per target."""
    arrs = [_f64(a) for a in (x, y, z, vx, vy, vz)]
    u = None if u is None else _f64(u)
    level = np.ascontiguousarray(level, dtype=np.int8)
    h, rho, omega = _f64(h), _f64(rho), _f64(omega)
    n = arrs[0].shape[0]
    tg = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    nt = n if tg is None else tg.shape[0]
    lo, hi = _box(lo, hi)
    out = {k: np.empty(nt) for k in ("ax", "ay", "az", "dudt", "vsig", "anorm", "unorm")}
    lib().orc_forces(n, *[_p(a, _d) for a in arrs], _p(u, _d), _p(level, _i8), _p(h, _d),
                     _p(rho, _d), _p(omega, _d), m0, eos, cs0, q_cs, r_ref, gamma, alpha,
                     beta, int(bool(periodic)), _p(lo, _d), _p(hi, _d), nt, _p(tg, _i64),
                     *[_p(out[k], _d) for k in ("ax", "ay", "az", "dudt", "vsig", "anorm",
                                                 "unorm")], int(kernel))
    return out


# ---------------------------------------------------------------- integration
def kick(vx, vy, vz, u, ax, ay, az, dudt, dt):
    """v += dt a, u += dt du/dt, in place."""
    n = vx.shape[0]
    lib().orc_kick(n, _p(vx, _d), _p(vy, _d), _p(vz, _d), _p(u, _d), _p(_f64(ax), _d),
                   _p(_f64(ay), _d), _p(_f64(az), _d),
                   None if dudt is None else _p(_f64(dudt), _d), dt)


def drift(x, y, z, vx, vy, vz, dt, *, periodic=False, lo=(0, 0, 0), hi=(1, 1, 1)):
    """x += dt v (wrapped into the box if periodic), in place."""
    lo, hi = _box(lo, hi)
    lib().orc_drift(x.shape[0], _p(x, _d), _p(y, _d), _p(z, _d), _p(_f64(vx), _d),
                    _p(_f64(vy), _d), _p(_f64(vz), _d), dt, int(bool(periodic)), _p(lo, _d),
                    _p(hi, _d))


def sink_gravity(x, y, z, sinks_x, sinks_m, sinks_eps, G, ax, ay, az):
    """Adds the point-mass gravity of the sinks to ax, ay, az in place."""
    sx = _f64(np.asarray(sinks_x).reshape(-1))
    sm, se = _f64(sinks_m), _f64(sinks_eps)
    lib().orc_sink_gravity(x.shape[0], _p(_f64(x), _d), _p(_f64(y), _d), _p(_f64(z), _d),
                           sm.shape[0], _p(sx, _d), _p(sm, _d), _p(se, _d), G, _p(ax, _d),
                           _p(ay, _d), _p(az, _d))


# ----------------------------------------------------------------------- APR
def splitmix64(state, k):
    """k-th SplitMix64 output (k >= 1) from the given state."""
    return int(lib().orc_splitmix64(C.c_uint64(state & (2**64 - 1)), C.c_uint64(k)))


def _zones_arrays(zones):
    nz = len(zones)
    zc = np.zeros((max(nz, 1), 3))
    zn = np.zeros(max(nz, 1), np.int32)
    zr = np.zeros((max(nz, 1), 8))
    ze = np.zeros((max(nz, 1), 8), np.int32)
    zs = np.zeros(max(nz, 1), np.int32)
    for k, zd in enumerate(zones):
        zc[k] = zd["c"]
        rr = list(zd["r"])
        ll = list(zd["ell"])
        zn[k] = len(rr)
        zr[k, :len(rr)] = rr
        ze[k, :len(ll)] = ll
        zs[k] = int(zd.get("shape", 0))
    return nz, zc, zn, zr, ze, zs


def zone_level(x, y, z, zones, background=0, derefine=False):
    """Refinement level at a point; a zone dict may set shape=1 (cylinders
    along z through c instead of spheres)."""
    nz, zc, zn, zr, ze, zs = _zones_arrays(zones)
    return int(lib().orc_zone_level(float(x), float(y), float(z), nz, _p(zc, _d),
                                    _p(zn, _i32), _p(zr, _d), _p(ze, _i32), _p(zs, _i32),
                                    background, int(bool(derefine))))


def pair_tree(cand, x, y, z, ids, lo, hi):
    """Leaf pairs of the merge pairing tree over particle indices cand."""
    cand = np.ascontiguousarray(cand, dtype=np.int64)
    x, y, z = _f64(x), _f64(y), _f64(z)
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    lo, hi = _box(lo, hi)
    n = x.shape[0]
    pairs = np.empty(max(n, 2), np.int64)
    np_ = lib().orc_pair_tree(cand.shape[0], _p(cand, _i64), _p(x, _d), _p(y, _d), _p(z, _d),
                              _p(ids, _i64), _p(lo, _d), _p(hi, _d), n, _p(pairs, _i64))
    return pairs[:2 * np_].reshape(-1, 2).copy()


def split_merge(st, zones, *, step, seed, r_sep_factor=0.2, nn_cap=0.35, split_mode=0,
                background=0, derefine=False, periodic=False, lo=(0, 0, 0), hi=(1, 1, 1),
                dnn=None, cap=None, do_split=True, do_merge=True, active=None):
    """One split/merge pass on a dict of numpy SoA arrays.

    st holds x, y, z, vx, vy, vz, u, h (float64), level (int8), id (int64) and
    next_id (int).  Returns a new dict (arrays trimmed to the new n) plus the
    counts n_split, n_merged, n_spare, origin (each particle's slot before the
    pass; an appended child's is its parent's) and changed (made by a split or
    kept by a merge).  active (bool [n], optional): only those particles split
    or pair for merging (individual timesteps, paper Sec. 2.5)."""
    n = st["x"].shape[0]
    cap = cap if cap is not None else 2 * n + 2
    w = {}
    for k in ("x", "y", "z", "vx", "vy", "vz", "u", "h"):
        a = np.zeros(cap)
        a[:n] = st[k]
        w[k] = a
    lev = np.zeros(cap, np.int8)
    lev[:n] = st["level"]
    ids = np.zeros(cap, np.int64)
    ids[:n] = st["id"]
    nid = C.c_int64(int(st["next_id"]))
    nz, zc, zn, zr, ze, zs = _zones_arrays(zones)
    lo, hi = _box(lo, hi)
    dn = None if dnn is None else _f64(dnn)
    act = None if active is None else np.ascontiguousarray(active, dtype=np.uint8)
    origin = np.zeros(cap, np.int64)
    changed = np.zeros(cap, np.uint8)
    n_out, ns, nm, nsp = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
    rc = lib().orc_split_merge(n, cap, *[_p(w[k], _d) for k in ("x", "y", "z", "vx", "vy", "vz",
                                                                 "u", "h")],
                               _p(lev, _i8), _p(ids, _i64), C.byref(nid), _p(dn, _d), nz,
                               _p(zc, _d), _p(zn, _i32), _p(zr, _d), _p(ze, _i32),
                               _p(zs, _i32), background,
                               int(bool(derefine)), r_sep_factor, nn_cap, split_mode,
                               C.c_uint64(seed & (2**64 - 1)), step, int(bool(periodic)),
                               _p(lo, _d), _p(hi, _d), int(bool(do_split)),
                               int(bool(do_merge)), C.byref(n_out), C.byref(ns), C.byref(nm),
                               C.byref(nsp), None if act is None else act.ctypes.data_as(_u8),
                               _p(origin, _i64), changed.ctypes.data_as(_u8))
    if rc != 0:
        raise RuntimeError("oracle split_merge: capacity %d too small, need %d" % (cap, ns.value))
    m = n_out.value
    out = {k: w[k][:m].copy() for k in w}
    out["level"] = lev[:m].copy()
    out["id"] = ids[:m].copy()
    out["next_id"] = nid.value
    out["n_split"], out["n_merged"], out["n_spare"] = ns.value, nm.value, nsp.value
    out["origin"] = origin[:m].copy()     # slot before the pass (children: the parent's)
    out["changed"] = changed[:m].astype(bool)
    return out


# -------------------------------------------------------------------- relaxing
def interp(tx, ty, tz, rx, ry, rz, rh, q, *, kernel=KERNEL_M4, periodic=False, lo=(0, 0, 0),
           hi=(1, 1, 1)):
    """The reference set's SPH interpolant sum_b q_b W(|x - x_b|, h_b) at the
    points (tx, ty, tz); q is [3, nr] (q_b = (m_b / rho_b) A_b)."""
    tx, ty, tz = _f64(tx), _f64(ty), _f64(tz)
    rx, ry, rz, rh = _f64(rx), _f64(ry), _f64(rz), _f64(rh)
    q = [_f64(q[k]) for k in range(3)]
    lo, hi = _box(lo, hi)
    nt, nr = tx.shape[0], rx.shape[0]
    out = [np.empty(nt) for _ in range(3)]
    lib().orc_interp(nt, _p(tx, _d), _p(ty, _d), _p(tz, _d), nr, _p(rx, _d), _p(ry, _d),
                     _p(rz, _d), _p(rh, _d), *[_p(a, _d) for a in q], int(kernel),
                     int(bool(periodic)), _p(lo, _d), _p(hi, _d), *[_p(a, _d) for a in out])
    return np.array(out)


_eos_fn = eos  # relax() takes the EOS kind under the name eos


def relax(st, ref, ref_rho, ref_a, *, m0, eos, hfact=1.2, kernel=KERNEL_M4, cs0=1.0, q_cs=0.25,
          r_ref=1.0, gamma=5.0 / 3.0, alpha=1.0, beta=2.0, periodic=False, lo=(0, 0, 0),
          hi=(1, 1, 1), max_shuffles=50, ke_frac=0.005, tol=1e-12):
    """Relaxing (paper Sec. 2.4) of the particles a split/merge pass introduced.

    st: the new set (dict of arrays, changed in place: x, y, z, h); ref: the
    reference set before the pass, with its converged densities ref_rho and
    accelerations ref_a [3, n_ref].  The shuffled particles are those with an id
    the reference does not hold (id >= ref next_id) or whose level differs
    from the reference's for the same id.  Each shuffle:
      1. a_new: hydro accelerations of the new set (density with its h-rho
         solve, then forces) at the current positions;
      2. a_ref: the reference accelerations interpolated at the same points;
      3. dx = 0.5 dt^2 (a_new - a_ref), dt = 0.3 h / c_s of the particle, its
         length capped at h; positions shift (periodic wrap);
      4. KE = sum |dx| / dt^2 over the shuffled particles.
    Repeats until KE <= ke_frac KE of the first shuffle, or max_shuffles.
    Returns (number of shuffles, list of KE)."""
    box = dict(periodic=periodic, lo=lo, hi=hi)
    lvl = {int(i): int(l) for i, l in zip(ref["id"], ref["level"])}
    nid = int(ref["next_id"])
    mask = np.array([int(i) >= nid or lvl.get(int(i), -1) != int(l)
                     for i, l in zip(st["id"], st["level"])])
    mref = m0 * 2.0 ** -ref["level"].astype(np.float64)
    q = (mref / ref_rho) * np.asarray(ref_a)
    lo_a, hi_a = np.asarray(lo, float), np.asarray(hi, float)
    L = hi_a - lo_a
    kes = []
    for k in range(max_shuffles):
        d = density(st["x"], st["y"], st["z"], st["level"], st["h"], m0=m0, hfact=hfact, tol=tol,
                    max_iter=60, kernel=kernel, **box)
        st["h"] = d["h"]
        f = forces(st["x"], st["y"], st["z"], st["vx"], st["vy"], st["vz"], st.get("u"),
                   st["level"], d["h"], d["rho"], d["omega"], m0=m0, eos=eos, cs0=cs0, q_cs=q_cs,
                   r_ref=r_ref, gamma=gamma, alpha=alpha, beta=beta, kernel=kernel, **box)
        aref = interp(st["x"], st["y"], st["z"], ref["x"], ref["y"], ref["z"], ref["h"], q,
                      kernel=kernel, **box)
        _, c = _eos_fn(st["x"], st["y"], d["rho"], st.get("u"), eos=eos, cs0=cs0, q_cs=q_cs,
                       r_ref=r_ref, gamma=gamma)
        anew = np.array([f["ax"], f["ay"], f["az"]])
        dt = 0.3 * d["h"] / c
        dx = 0.5 * dt * dt * (anew - aref)
        ln = np.sqrt((dx * dx).sum(0))
        big = ln > d["h"]
        dx[:, big] *= d["h"][big] / ln[big]
        ln = np.minimum(ln, d["h"])
        dx[:, ~mask] = 0.0
        for a, key in enumerate(("x", "y", "z")):
            v = st[key] + dx[a]
            if periodic:  # one image back into [lo, hi), as the drift does
                v = np.where(v >= hi_a[a], v - L[a], np.where(v < lo_a[a], v + L[a], v))
            st[key] = v
        kes.append(float(np.sum((ln / (dt * dt))[mask])))
        if kes[-1] <= ke_frac * kes[0]:
            break
    return len(kes), kes


# ------------------------------------------------------- individual timesteps
def courant_bin(h, vsig, *, dt_max, c_cfl, max_bin):
    """Timestep bin from the Courant limit dt_C = c_cfl h / vsig: the smallest
    k >= 0 with dt_max 2^-k <= dt_C, at most max_bin (an integer search, so
    that the decision is exact)."""
    dtc = c_cfl * np.asarray(h, float) / np.asarray(vsig, float)
    k = np.zeros(dtc.shape[0], np.int8)
    for b in range(max_bin):
        k += (k == b) & (np.ldexp(dt_max, -b) > dtc)
    return k


_PERSIST = ("rho", "omega", "ax", "ay", "az", "dudt", "vsig", "dnn", "bin")


def accel_bins(st, *, m0, eos, hfact=1.2, kernel=KERNEL_M4, cs0=1.0, q_cs=0.25, r_ref=1.0,
               gamma=5.0 / 3.0, alpha=1.0, beta=2.0, periodic=False, lo=(0, 0, 0),
               hi=(1, 1, 1), sinks=(), G=1.0, targets=None, tol=1e-12):
    """Density (h-rho solve), forces and sink gravity for the targets (all if
    None), stored in st: h, rho, omega, dnn, ax, ay, az, dudt, vsig.  The
    other particles keep their stored values, which their neighbours use."""
    n = st["x"].shape[0]
    idx = np.arange(n) if targets is None else np.asarray(targets, np.int64)
    if idx.size == 0:
        return
    box = dict(periodic=periodic, lo=lo, hi=hi)
    d = density(st["x"], st["y"], st["z"], st["level"], st["h"][idx], m0=m0, hfact=hfact,
                tol=tol, max_iter=60, kernel=kernel, targets=idx, **box)
    for k in ("rho", "omega", "dnn"):
        if k not in st:
            st[k] = np.ones(n)
    st["h"][idx], st["rho"][idx], st["omega"][idx], st["dnn"][idx] = (
        d["h"], d["rho"], d["omega"], d["dnn"])
    f = forces(st["x"], st["y"], st["z"], st["vx"], st["vy"], st["vz"], st.get("u"),
               st["level"], st["h"], st["rho"], st["omega"], m0=m0, eos=eos, cs0=cs0,
               q_cs=q_cs, r_ref=r_ref, gamma=gamma, alpha=alpha, beta=beta, kernel=kernel,
               targets=idx, **box)
    if sinks:
        sink_gravity(st["x"][idx], st["y"][idx], st["z"][idx], [s_["x"] for s_ in sinks],
                     [s_["m"] for s_ in sinks], [s_.get("eps", 0.0) for s_ in sinks], G,
                     f["ax"], f["ay"], f["az"])
    for k in ("ax", "ay", "az", "dudt", "vsig"):
        if k not in st:
            st[k] = np.zeros(n)
        st[k][idx] = f[k]


def step_bins(st, *, zones, dt_max, step, max_bin, c_cfl=0.3, seed=0, r_sep_factor=0.2,
              nn_cap=0.35, split_mode=0, **phys):
    """One step of length dt_max with individual timesteps (paper Sec. 2.5).

    st holds the state and, per particle, bin (int8) and the stored rho, omega,
    dnn, ax, ay, az, dudt, vsig of its last evaluation (accel_bins).  Bin k
    steps with dt_max 2^-k; K = max bin, 2^K substeps of dt_max 2^-K.  In
    substep s a particle whose step starts (s a multiple of 2^(K-k)) takes its
    opening half kick (v, and u if adiabatic, with its own dt); every
    particle drifts; the particles whose step ends ((s+1) a multiple of
    2^(K-k)) are active: the split/merge pass examines only them (random key
    step 4096 + s), density, forces and sink gravity are taken for them (and
    for what the pass made), they take their closing half kick, and their bin
    follows the Courant limit, clamped to K within the step (the substep grid
    is fixed) and to max_bin at its end, lengthened only where the longer step
    starts at this boundary; what the pass made or kept takes bin K.
    Returns the new state dict."""
    box = dict(periodic=phys.get("periodic", False), lo=phys.get("lo", (0, 0, 0)),
               hi=phys.get("hi", (1, 1, 1)))
    adiab = phys["eos"] == EOS_ADIABATIC
    st = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()}
    K = int(st["bin"].max())
    nsub = 1 << K
    delta = np.ldexp(dt_max, -K)
    for s in range(nsub):
        b = st["bin"].astype(np.int64)
        stride = np.left_shift(1, K - b)
        dta = np.ldexp(dt_max, -b)
        op = (s % stride) == 0
        for v, a in (("vx", "ax"), ("vy", "ay"), ("vz", "az")) + ((("u", "dudt"),) if adiab else ()):
            st[v][op] += 0.5 * dta[op] * st[a][op]
        drift(st["x"], st["y"], st["z"], st["vx"], st["vy"], st["vz"], delta, **box)
        act = ((s + 1) % stride) == 0
        if zones:
            out = split_merge(st, zones, step=step * 4096 + s, seed=seed,
                              r_sep_factor=r_sep_factor, nn_cap=nn_cap, split_mode=split_mode,
                              dnn=st["dnn"], active=act, **box)
            o = out["origin"]
            new = {k: out[k] for k in ("x", "y", "z", "vx", "vy", "vz", "u", "h", "level", "id",
                                       "next_id")}
            for k in _PERSIST:
                new[k] = st[k][o].copy()
            act = act[o] | out["changed"]
            made = out["changed"]
            st = new
        else:
            made = np.zeros(st["x"].shape[0], bool)
        idx = np.nonzero(act)[0]
        accel_bins(st, targets=idx, **phys)
        b = st["bin"].astype(np.int64)
        dta = np.ldexp(dt_max, -b)
        for v, a in (("vx", "ax"), ("vy", "ay"), ("vz", "az")) + ((("u", "dudt"),) if adiab else ()):
            st[v][act] += 0.5 * dta[act] * st[a][act]
        last = s + 1 == nsub
        kc = courant_bin(st["h"], st["vsig"], dt_max=dt_max, c_cfl=c_cfl,
                         max_bin=max_bin if last else K).astype(np.int64)
        for i in idx:
            k = K if made[i] else int(kc[i])
            while not last and (s + 1) % (1 << (K - k)):
                k += 1
            st["bin"][i] = k
    return st
