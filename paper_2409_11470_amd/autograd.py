"""torch.autograd.Function over the density and force sums.

apr_sums(ctx, st, x, y, z, m) runs apr_build_cells, apr_density and
apr_forces on a private copy of the state st with positions (x, y, z) and
returns (rho, h, ax, ay, az, dudt) in the particle order of the inputs.  Its
backward is apr_vjp: the implicit h, the EOS and the grad-h Omega are
differentiated in the library (neighbours are searched again).  m is the
gradient handle of the masses m_a = m0 2^-level_a (its values are not read:
the library takes masses from the levels); velocities, u and the levels are
held fixed.
"""
import torch

from . import api


class _Sums(torch.autograd.Function):
    @staticmethod
    def forward(fctx, x, y, z, m, actx, st):
        w = st.clone()
        n = w.n
        dev = w.t["x"].device
        with torch.no_grad():
            w.t["x"][:n].copy_(x)
            w.t["y"][:n].copy_(y)
            w.t["z"][:n].copy_(z)
        perm = torch.empty(n, dtype=torch.int64, device=dev)
        api.apr_build_cells(actx, w, perm)
        dt = actx.dtype
        rho = torch.empty(n, dtype=dt, device=dev)
        om = torch.empty(n, dtype=dt, device=dev)
        api.apr_density(actx, w, rho, om)
        api.apr_sync_status(actx)
        acc = [torch.empty(n, dtype=dt, device=dev) for _ in range(4)]
        api.apr_forces(actx, w, rho, om, *acc)
        outs = []
        for t in [rho, w.t["h"][:n].to(dt)] + acc:
            o = torch.empty_like(t)
            o[perm] = t
            outs.append(o)
        fctx.save_for_backward(perm, rho, om)
        fctx.actx, fctx.w = actx, w
        fctx.in_dtype = x.dtype
        fctx.mark_non_differentiable()
        return tuple(outs)

    @staticmethod
    def backward(fctx, grho, gh, gax, gay, gaz, gdu):
        perm, rho, om = fctx.saved_tensors
        actx, w = fctx.actx, fctx.w
        # the cells may have been replaced by another call on this context;
        # the copy is already in Morton order, so this is cheap
        p2 = torch.empty_like(perm)
        api.apr_build_cells(actx, w, p2)
        perm, rho, om = perm[p2], rho[p2], om[p2]
        dt = actx.dtype

        def srt(g):
            return None if g is None else g.to(dt)[perm].contiguous()

        xb, yb, zb, mb = api.apr_vjp(actx, w, rho, om, srt(grho), srt(gh), srt(gax), srt(gay),
                                     srt(gaz), srt(gdu))
        res = []
        for t in (xb, yb, zb, mb):
            o = torch.empty(t.shape, dtype=fctx.in_dtype, device=t.device)
            o[perm] = t.to(fctx.in_dtype)
            res.append(o)
        return res[0], res[1], res[2], res[3], None, None


def apr_sums(ctx, st, x=None, y=None, z=None, m=None):
    """(rho, h, ax, ay, az, dudt) with gradients to x, y, z [n] and m [n]."""
    n = st.n
    x = st["x"] if x is None else x
    y = st["y"] if y is None else y
    z = st["z"] if z is None else z
    if m is None:
        m = ctx.params.m0 * torch.pow(2.0, -st["level"].double())
    return _Sums.apply(x, y, z, m, ctx, st)
