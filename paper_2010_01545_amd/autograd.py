"""torch.autograd.Function over the library's forward and gather adjoint.

``PWAdvect.apply(u, v, w, tzc1, tzc2, tcx, tcy, halo, compute)`` takes interior
tensors (nx, ny, nz) of a domain periodic in x and y, pads them with the
library's periodic halo kernel, runs the forward kernel and returns the
interior source terms (su, sv, sw).  Backward pads the incoming gradients the
same way and runs the adjoint kernel, which re-reads the (padded) winds
instead of storing any intermediate.  The coefficients get no gradient.
``compute=torch.float64`` with float32 tensors selects FP64 arithmetic on
float storage for both passes.
"""
import torch

from . import pwadvect


class PWAdvect(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, v, w, tzc1, tzc2, tcx, tcy, halo=2, compute=None):
        h = int(halo)
        st = [pwadvect.pad_periodic(t.contiguous(), h) for t in (u, v, w)]
        tzc1, tzc2 = (torch.as_tensor(t, dtype=torch.float64, device=u.device).contiguous()
                      for t in (tzc1, tzc2))
        su, sv, sw = pwadvect.fwd(*st, tzc1, tzc2, tcx, tcy, h, compute=compute)
        ctx.save_for_backward(*st, tzc1, tzc2)
        ctx.tcx, ctx.tcy, ctx.h, ctx.compute = tcx, tcy, h, compute
        return tuple(s[h:-h, h:-h, h:-h] for s in (su, sv, sw))

    @staticmethod
    def backward(ctx, gsu, gsv, gsw):
        us, vs, ws, tzc1, tzc2 = ctx.saved_tensors
        h = ctx.h
        lam = []
        for g in (gsu, gsv, gsw):
            if g is None:
                g = torch.zeros(tuple(n - 2 * h for n in us.shape), dtype=us.dtype, device=us.device)
            lam.append(pwadvect.pad_periodic(g.contiguous(), h))
        gu, gv, gw = pwadvect.adj(us, vs, ws, *lam, tzc1, tzc2, ctx.tcx, ctx.tcy, h, compute=ctx.compute)
        return (gu[h:-h, h:-h, h:-h], gv[h:-h, h:-h, h:-h], gw[h:-h, h:-h, h:-h],
                None, None, None, None, None, None)


def pw_advect(u, v, w, tzc1, tzc2, tcx, tcy, halo=2, compute=None):
    """Functional form of PWAdvect.apply."""
    return PWAdvect.apply(u, v, w, tzc1, tzc2, tcx, tcy, halo, compute)
