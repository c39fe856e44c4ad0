"""The launch grid of the per-cell kernels is an implementation setting.

The cell count stays on the device; the host sizes the grids from an estimate
and a second launch of each search kernel takes any cells beyond the grid
(which also lie beyond the candidate lists' capacity, so those cells walk the
tree themselves).  With a grid far below the cell count every result must be
bit-identical to the default grid's: each cell is computed by one workgroup
whichever workgroup it is, in the same order."""
import numpy as np
import pytest
import torch

import paper_2409_11470_amd as A
import workloads as W
from _gpu import params_for

pytestmark = pytest.mark.gpu


def _run(st, p, prec, grid):
    ctx = A.Context(params_for(p, prec))
    if grid:
        A.apr_set_cell_grid(ctx, grid)
    ds = A.DeviceState.from_numpy(st)
    A.apr_build_cells(ctx, ds)
    n = ds.n
    dt = ctx.dtype
    rho = torch.zeros(n, dtype=dt, device="cuda")
    om = torch.zeros(n, dtype=dt, device="cuda")
    nn = torch.zeros(n, dtype=torch.int32, device="cuda")
    it = torch.zeros(n, dtype=torch.int32, device="cuda")
    A.apr_density(ctx, ds, rho, om, nn, it)
    out = {k: torch.zeros(n, dtype=dt, device="cuda") for k in ("ax", "ay", "az", "dudt", "vsig")}
    A.apr_forces(ctx, ds, rho, om, out["ax"], out["ay"], out["az"], out["dudt"], out["vsig"])
    g = torch.Generator(device="cpu").manual_seed(5)
    cot = {k: torch.randn(n, generator=g, dtype=torch.float64).to("cuda").to(dt)
           for k in ("rho_bar", "h_bar", "ax_bar", "ay_bar", "az_bar", "dudt_bar")}
    xb, yb, zb, mb = A.apr_vjp(ctx, ds, rho, om, **cot)
    counts = A.apr_neighbours(ctx, ds, ds["h"], mode=1, count_only=True)
    A.apr_sync_status(ctx)
    res = dict(h=ds["h"], rho=rho, om=om, nn=nn, it=it, xb=xb, yb=yb, zb=zb, mb=mb,
               counts=counts, **out)
    return {k: (v.cpu().numpy() if torch.is_tensor(v) else np.asarray(v)) for k, v in res.items()}


@pytest.mark.parametrize("prec", [
    "fp32",
    pytest.param("fp64", marks=pytest.mark.skip(
        reason="a GPU memory fault (aperture violation) in the FP64 force kernel's "
               "beyond-grid launch was seen once in this case with a build whose list "
               "building took two blocks of entries per step; that change is taken out, "
               "the cause is not shown, so the case stays off the GPU until it is")),
])
def test_small_grid_bit_identical(prec):
    st, p = W.lattice_box(nside=24)
    ref = _run(st, p, prec, 0)
    for grid in (1, 7):
        got = _run(st, p, prec, grid)
        for k in ref:
            assert np.array_equal(got[k], ref[k]), (grid, k)


def test_grid_setting_rejects_negative():
    ctx = A.Context(params_for(dict(m0=1.0), "fp32"))
    with pytest.raises(A.AprError):
        A.apr_set_cell_grid(ctx, -1)


def test_steps_grid_independent():
    """Steps size their grids from the count read back asynchronously at an
    earlier build; a grid of n (never short) and a grid of 5 (nearly all cells
    in the second launch) must give the same bits over several steps."""
    st, p = W.shock_box(nside=32)
    n = st["x"].shape[0]
    outs = []
    for grid in (0, n, 5):
        ctx = A.Context(params_for(p, "fp32"))
        if grid:
            A.apr_set_cell_grid(ctx, grid)
        ds = A.DeviceState.from_numpy(st)
        A.apr_accel(ctx, ds)
        dt = A.apr_timestep(ctx, ds, 0.3)
        for k in range(4):
            A.apr_step(ctx, ds, [], [], dt, k)
        A.apr_sync_status(ctx)
        outs.append(ds.to_numpy())
    for o in outs[1:]:
        for k in ("x", "y", "z", "vx", "vy", "vz", "u", "h", "id"):
            assert np.array_equal(o[k], outs[0][k]), k
