"""Neighbour lists for a given h: the GPU's exact FP64 predicate against the
oracle's brute force, compared as sorted id sets (bit-exact membership)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2409_11470_amd as A
import workloads as W
from _gpu import params_for

pytestmark = pytest.mark.gpu


def _gpu_lists(st, p, h, mode):
    ctx = A.Context(params_for(p, "fp64"))
    ds = A.DeviceState.from_numpy(st)
    A.apr_build_cells(ctx, ds)
    ids = ds["id"].cpu().numpy()
    hd = torch.from_numpy(h[ids]).cuda()
    offs, lst = A.apr_neighbours(ctx, ds, hd, mode)
    A.apr_sync_status(ctx)
    offs, lst = offs.cpu().numpy(), lst.cpu().numpy()
    out = [None] * ids.shape[0]
    for s in range(ids.shape[0]):
        out[ids[s]] = np.sort(ids[lst[offs[s]:offs[s + 1]]])
    return out


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("wl", ["lattice", "shock", "disc"])
def test_lists_bit_exact(mode, wl):
    if wl == "lattice":
        st, p = W.lattice_box()
    elif wl == "shock":
        st, p = W.shock_box(nside=20)
        p = dict(p, m0=1.0 / 20 ** 3)
    else:
        st, p = W.planet_disc(n=15000)
    o = oracle.density(st["x"], st["y"], st["z"], st["level"], st["h"], m0=p["m0"],
                       periodic=p["periodic"], lo=p["lo"], hi=p["hi"])
    h = o["h"]
    ref = oracle.neighbours(st["x"], st["y"], st["z"], h, symmetric=bool(mode),
                            periodic=p["periodic"], lo=p["lo"], hi=p["hi"])
    got = _gpu_lists(st, p, h, mode)
    for a in range(len(ref)):
        assert np.array_equal(got[a], ref[a]), a
