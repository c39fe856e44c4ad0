"""The allocation-free entry point apr_timestep_noalloc (for callers that
cannot allocate) against apr_timestep, through the C ABI: the Courant
timestep C min h / vsig of the same state, bit for bit, on two calls in a
row, the second with a smaller state (the library's per-GPU scratch keeps
the first call's partial minima; the second must read only its own), and
the argument errors."""
import ctypes as C

import numpy as np
import pytest
import torch

import paper_2409_11470_amd as A
import workloads as W
from _gpu import params_for

pytestmark = pytest.mark.gpu


def test_noalloc_timestep_matches_apr_timestep():
    lib = A.lib()
    # 68^3 = 314432 particles: more than 1024 blocks of 256, so the reduction
    # strides; then 12^3 = 1728 particles, 7 partial minima
    for nside in (68, 12):
        st, p = W.shock_box(nside=nside)
        p = dict(p, m0=1.0 / nside ** 3)
        for prec in ("fp32", "fp64"):
            ctx = A.Context(params_for(p, prec))
            ds = A.DeviceState.from_numpy(st)
            A.apr_accel(ctx, ds)
            ref = A.apr_timestep(ctx, ds, 0.3)
            out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
            cs = ds.cstate()
            rc = lib.apr_timestep_noalloc(ctx.ptr, C.byref(cs), C.c_double(0.3),
                                          C.c_void_p(out.data_ptr()))
            assert rc == A.APR_OK
            torch.cuda.synchronize()
            got = float(out.cpu().item())
            assert got == ref, (nside, prec, got, ref)
            assert np.isfinite(got) and got > 0.0
            ctx.close()


def test_noalloc_timestep_argument_errors():
    lib = A.lib()
    st, p = W.shock_box(nside=12)
    p = dict(p, m0=1.0 / 12 ** 3)
    ctx = A.Context(params_for(p, "fp32"))
    ds = A.DeviceState.from_numpy(st)
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    cs = ds.cstate()
    # no force evaluation of this state yet
    rc = lib.apr_timestep_noalloc(ctx.ptr, C.byref(cs), C.c_double(0.3),
                                  C.c_void_p(out.data_ptr()))
    assert rc == A.APR_ERR_INVALID
    A.apr_accel(ctx, ds)
    cs = ds.cstate()
    rc = lib.apr_timestep_noalloc(ctx.ptr, C.byref(cs), C.c_double(0.3), None)
    assert rc == A.APR_ERR_INVALID
    torch.cuda.synchronize()
    assert out.item() == 0.0  # nothing was written
    ctx.close()
