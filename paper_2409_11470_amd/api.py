"""Python binding of libapr.so with the C ABI's names.

Arguments are marshalled from torch tensors (device memory) and plain Python
values; every computation runs in the library.  Each apr_* function raises
AprError when the C call returns a non-zero status.
"""
import ctypes as C

import numpy as np
import torch

from ._abi import (APR_PROF_N, AprError, CState, Params, Sink, Zone, apr_default_params,
                   lib)

_DFIELDS = ("x", "y", "z", "vx", "vy", "vz", "u", "h", "ax", "ay", "az", "dudt")


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return C.c_void_p(t.data_ptr())


def _stream_handle():
    return torch.cuda.current_stream().cuda_stream


def make_params(**kw):
    """apr_params with the library defaults, overridden by keyword values."""
    p = apr_default_params()
    for k, v in kw.items():
        if k in ("box_lo", "box_hi"):
            getattr(p, k)[:] = [float(a) for a in v]
        elif k == "seed":
            p.seed = int(v) & (2 ** 64 - 1)
        elif not hasattr(p, k):
            raise KeyError(k)
        else:
            setattr(p, k, v)
    return p


def make_zones(zones):
    """ctypes array of apr_zone from dicts {c: (x, y, z), r: radii outer->inner,
    ell: levels, shape: 0 spheres (default) or 1 cylinders along z}."""
    arr = (Zone * max(1, len(zones)))()
    for k, z in enumerate(zones):
        arr[k].c[:] = [float(v) for v in z["c"]]
        r, e = list(z["r"]), list(z["ell"])
        if not 1 <= len(r) <= 8 or len(e) != len(r):
            raise ValueError("a zone has 1..8 spheres")
        arr[k].n = len(r)
        arr[k].shape = int(z.get("shape", 0))
        for i in range(len(r)):
            arr[k].r[i] = float(r[i])
            arr[k].ell[i] = int(e[i])
    return arr, len(zones)


def make_sinks(sinks):
    arr = (Sink * max(1, len(sinks)))()
    for k, s in enumerate(sinks):
        arr[k].x[:] = [float(v) for v in s["x"]]
        arr[k].m = float(s["m"])
        arr[k].eps = float(s.get("eps", 0.0))
    return arr, len(sinks)


class Context:
    """Owns an apr_ctx bound to the current torch stream."""

    def __init__(self, params, stream=None):
        if isinstance(params, dict):
            params = make_params(**params)
        self.params = params
        self.ptr = C.c_void_p()
        h = _stream_handle() if stream is None else stream
        rc = lib().apr_ctx_create(C.byref(self.ptr), C.byref(params), C.c_void_p(h))
        if rc != 0:
            raise AprError(rc, "apr_ctx_create failed")

    @property
    def fp32(self):
        return self.params.precision == 1

    @property
    def dtype(self):
        return torch.float32 if self.fp32 else torch.float64

    def error(self):
        return lib().apr_last_error(self.ptr).decode()

    def check(self, rc):
        if rc != 0:
            raise AprError(rc, self.error())

    def close(self):
        if self.ptr:
            lib().apr_ctx_destroy(self.ptr)
            self.ptr = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DeviceState:
    """Particle arrays on the GPU (structure of arrays) with room for `capacity`."""

    def __init__(self, capacity, device="cuda"):
        self.capacity = int(capacity)
        self.n = 0
        self.next_id = 0
        self.t = {k: torch.zeros(self.capacity, dtype=torch.float64, device=device)
                  for k in _DFIELDS}
        self.t["level"] = torch.zeros(self.capacity, dtype=torch.int8, device=device)
        self.t["id"] = torch.zeros(self.capacity, dtype=torch.int64, device=device)
        self.t["bin"] = torch.zeros(self.capacity, dtype=torch.int8, device=device)  # timestep bins

    @classmethod
    def from_numpy(cls, st, capacity=None, device="cuda"):
        n = st["x"].shape[0]
        self = cls(capacity or n, device)
        for k in ("x", "y", "z", "vx", "vy", "vz", "u", "h"):
            self.t[k][:n] = torch.from_numpy(np.ascontiguousarray(st[k], np.float64))
        self.t["level"][:n] = torch.from_numpy(np.ascontiguousarray(st["level"], np.int8))
        self.t["id"][:n] = torch.from_numpy(np.ascontiguousarray(st["id"], np.int64))
        self.n = n
        self.next_id = int(st.get("next_id", n))
        return self

    def to_numpy(self):
        n = self.n
        out = {k: v[:n].cpu().numpy() for k, v in self.t.items()}
        out["next_id"] = self.next_id
        return out

    def __getitem__(self, k):
        return self.t[k][:self.n]

    def cstate(self, with_accel=True):
        cs = CState()
        cs.n, cs.capacity, cs.next_id = self.n, self.capacity, self.next_id
        for k in _DFIELDS:
            if not with_accel and k in ("ax", "ay", "az", "dudt"):
                continue
            setattr(cs, k, self.t[k].data_ptr())
        cs.level = self.t["level"].data_ptr()
        cs.id = self.t["id"].data_ptr()
        return cs

    def absorb(self, cs):
        self.n = int(cs.n)
        self.next_id = int(cs.next_id)

    def clone(self):
        """A copy of the first n particles (capacity n)."""
        c = DeviceState.__new__(DeviceState)
        c.capacity, c.n, c.next_id = max(1, self.n), self.n, self.next_id
        c.t = {k: v[:c.capacity].clone() for k, v in self.t.items()}
        return c

    def grow(self, capacity):
        if capacity <= self.capacity:
            return
        for k, v in self.t.items():
            nv = torch.zeros(capacity, dtype=v.dtype, device=v.device)
            nv[:self.n] = v[:self.n]
            self.t[k] = nv
        self.capacity = int(capacity)


# ----------------------------------------------------------- C-ABI functions
def apr_ctx_create(params, stream=None):
    return Context(params, stream)


def apr_ctx_destroy(ctx):
    ctx.close()


def apr_set_cell_grid(ctx, grid):
    ctx.check(lib().apr_set_cell_grid(ctx.ptr, int(grid)))


def apr_build_cells(ctx, st, perm=None):
    cs = st.cstate()
    ctx.check(lib().apr_build_cells(ctx.ptr, C.byref(cs), _ptr(perm)))


def apr_density(ctx, st, rho, omega, nneigh=None, iters=None):
    cs = st.cstate()
    ctx.check(lib().apr_density(ctx.ptr, C.byref(cs), _ptr(rho), _ptr(omega), _ptr(nneigh),
                                _ptr(iters)))


def apr_forces(ctx, st, rho, omega, ax, ay, az, dudt, vsig=None, npair=None):
    cs = st.cstate()
    ctx.check(lib().apr_forces(ctx.ptr, C.byref(cs), _ptr(rho), _ptr(omega), _ptr(ax), _ptr(ay),
                               _ptr(az), _ptr(dudt), _ptr(vsig), _ptr(npair)))


def apr_vjp(ctx, st, rho, omega, rho_bar=None, h_bar=None, ax_bar=None, ay_bar=None,
            az_bar=None, dudt_bar=None):
    """Adjoint of apr_density + apr_forces on the current cells: returns
    (xbar, ybar, zbar, mbar), device tensors of the context precision."""
    n = st.n
    out = [torch.empty(n, dtype=ctx.dtype, device=rho.device) for _ in range(4)]
    cs = st.cstate()
    ctx.check(lib().apr_vjp(ctx.ptr, C.byref(cs), _ptr(rho), _ptr(omega), _ptr(rho_bar),
                            _ptr(h_bar), _ptr(ax_bar), _ptr(ay_bar), _ptr(az_bar),
                            _ptr(dudt_bar), *[_ptr(t) for t in out]))
    return tuple(out)


def apr_bins_init(ctx, st, dt_max, c_cfl=0.3, max_bin=8, sinks=()):
    """Individual timesteps: accelerations of every particle and its Courant
    bin (st["bin"])."""
    sarr, ns = make_sinks(list(sinks))
    cs = st.cstate()
    ctx.check(lib().apr_bins_init(ctx.ptr, C.byref(cs), _ptr(st.t["bin"]), sarr, ns,
                                  float(dt_max), float(c_cfl), int(max_bin)))


def apr_step_bins(ctx, st, zones, sinks, dt_max, step, c_cfl=0.3, max_bin=8):
    """One step of dt_max with individual timesteps; returns the number of
    substeps.  With zones the state first gets room for two splits per
    particle."""
    zarr, nz = make_zones(zones)
    sarr, ns = make_sinks(list(sinks))
    if nz > 0:
        st.grow(3 * st.n + 64)
    cs = st.cstate()
    nsub = C.c_int32()
    ctx.check(lib().apr_step_bins(ctx.ptr, C.byref(cs), _ptr(st.t["bin"]), zarr, nz, sarr, ns,
                                  float(dt_max), float(c_cfl), int(max_bin), int(step),
                                  C.byref(nsub)))
    st.absorb(cs)
    return nsub.value


def apr_relax(ctx, st, ref_ctx, ref, ref_rho, ref_ax, ref_ay, ref_az, max_shuffles=50,
              ke_frac=0.005):
    """Relaxing (paper Sec. 2.4) of the particles of st that a split/merge pass
    introduced, against the reference state ref (the state before the pass,
    with cells built in ref_ctx and ref_rho, ref_a* from apr_density and
    apr_forces there).  Returns (shuffles, first KE, last KE)."""
    cs, rcs = st.cstate(), ref.cstate()
    ns, k0, k1 = C.c_int32(), C.c_double(), C.c_double()
    ctx.check(lib().apr_relax(ctx.ptr, C.byref(cs), ref_ctx.ptr, C.byref(rcs), _ptr(ref_rho),
                              _ptr(ref_ax), _ptr(ref_ay), _ptr(ref_az), int(max_shuffles),
                              float(ke_frac), C.byref(ns), C.byref(k0), C.byref(k1)))
    return ns.value, k0.value, k1.value


def apr_neighbours(ctx, st, h, mode=0, count_only=False):
    """Neighbour slots per particle for the given h (device float64 [n]).
    Returns (offsets [n+1], list) as device int64 tensors, or only the total
    number of pairs if count_only."""
    n = st.n
    dev = h.device
    counts = torch.zeros(n, dtype=torch.int64, device=dev)
    offs = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    total = C.c_int64()
    cs = st.cstate()
    ctx.check(lib().apr_neighbours(ctx.ptr, C.byref(cs), _ptr(h), mode, _ptr(counts),
                                   _ptr(offs), None, 0, C.byref(total)))
    if count_only:
        return int(total.value)
    lst = torch.zeros(max(1, total.value), dtype=torch.int64, device=dev)
    ctx.check(lib().apr_neighbours(ctx.ptr, C.byref(cs), _ptr(h), mode, _ptr(counts),
                                   _ptr(offs), _ptr(lst), lst.numel(), C.byref(total)))
    return offs, lst[:total.value]


def apr_split_merge(ctx, st, zones, step, flags=0):
    """One split/merge pass; grows st if the splits need room.  Returns
    (n_split, n_merged, n_spare)."""
    zarr, nz = make_zones(zones)
    while True:
        cs = st.cstate()
        ns, nm, nsp = C.c_int64(), C.c_int64(), C.c_int64()
        rc = lib().apr_split_merge(ctx.ptr, C.byref(cs), zarr, nz, int(step), int(flags),
                                   C.byref(ns), C.byref(nm), C.byref(nsp))
        if rc == 2:  # APR_ERR_CAPACITY: grow and retry
            st.grow(int(ns.value * 5 // 4) + 64)
            continue
        ctx.check(rc)
        st.absorb(cs)
        return ns.value, nm.value, nsp.value


def apr_step(ctx, st, zones, sinks, dt, step):
    zarr, nz = make_zones(zones)
    sarr, ns = make_sinks(sinks)
    if nz > 0:
        # room for the worst case of this pass (every particle splits)
        st.grow(2 * st.n + 64)
    cs = st.cstate()
    rc = lib().apr_step(ctx.ptr, C.byref(cs), zarr, nz, sarr, ns, float(dt), int(step))
    ctx.check(rc)
    st.absorb(cs)


def apr_accel(ctx, st, sinks=()):
    sarr, ns = make_sinks(list(sinks))
    cs = st.cstate()
    ctx.check(lib().apr_accel(ctx.ptr, C.byref(cs), sarr, ns))


def apr_timestep(ctx, st, C_cfl=0.3):
    dt = C.c_double()
    cs = st.cstate()
    ctx.check(lib().apr_timestep(ctx.ptr, C.byref(cs), float(C_cfl), C.byref(dt)))
    return dt.value


def apr_timestep_noalloc(ctx, st, dt_dev, C_cfl=0.3):
    """apr_timestep into a device float64 tensor of one element, with no
    allocation and no synchronisation (enqueued on the context's stream)."""
    cs = st.cstate()
    ctx.check(lib().apr_timestep_noalloc(ctx.ptr, C.byref(cs), float(C_cfl), _ptr(dt_dev)))


def apr_sync_status(ctx, raise_noconverge=True):
    """Waits for the stream; returns the number of unconverged h-rho solves.
    Raises AprError on any flag (non-convergence only if raise_noconverge)."""
    cnt = C.c_int64()
    rc = lib().apr_sync_status(ctx.ptr, C.byref(cnt))
    if rc == 3 and not raise_noconverge:
        return cnt.value
    if rc != 0:
        raise AprError(rc, ctx.error())
    return cnt.value


def apr_profile_enable(ctx, on=True):
    ctx.check(lib().apr_profile_enable(ctx.ptr, int(bool(on))))


def apr_profile_select(ctx, indices=None):
    """Times only the given APR_PROF_* indices (None: all of them)."""
    mask = 0xFFFFFFFF if indices is None else sum(1 << int(k) for k in indices)
    ctx.check(lib().apr_profile_select(ctx.ptr, mask))


def apr_profile_read(ctx, reset=True):
    """{index: (total ms, launches)} for the timed kernels; synchronises."""
    ms = (C.c_double * APR_PROF_N)()
    cnt = (C.c_int64 * APR_PROF_N)()
    ctx.check(lib().apr_profile_read(ctx.ptr, ms, cnt, int(bool(reset))))
    return {k: (ms[k], cnt[k]) for k in range(APR_PROF_N)}


COUNTER_NAMES = ("noconverge", "periodic_range", "density_multiwindow_cells",
                 "force_multiwindow_cells", "subblock_direct", "density_restage",
                 "density_passes", "density_windows", "band_beyond_slack", "edge_tests")


def apr_counters(ctx, reset=True):
    """Work counters (see include/apr.h) as a dict; synchronises."""
    c = (C.c_int64 * len(COUNTER_NAMES))()
    ctx.check(lib().apr_counters(ctx.ptr, c, int(bool(reset))))
    return {k: int(c[i]) for i, k in enumerate(COUNTER_NAMES)}
