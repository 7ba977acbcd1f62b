"""The oracle's scatter adjoint against torch autograd (CPU, float64).

The source terms are written a second time with whole-array torch slicing
(section 2.1, Listing 1, and the sv/sw readings), the periodic x/y halo fill
is a differentiable wrap, and autograd differentiates
L = sum(lu*su + lv*sv + lw*sw) over interior cells.  The adjoint that autograd
derives is independent of the oracle's hand-written term-by-term scatter and
periodic fold.
"""
import numpy as np
import torch

from paper_2010_01545_amd import inputs

H = 1


def _pad(x):
    """Interior (nx, ny, nz) -> storage with halo H: periodic in x and y, zero in z."""
    x = torch.cat([x[-H:], x, x[:H]], dim=0)
    x = torch.cat([x[:, -H:], x, x[:, :H]], dim=1)
    z = torch.zeros(x.shape[0], x.shape[1], H, dtype=x.dtype)
    return torch.cat([z, x, z], dim=2)


def _fwd_torch(u, v, w, tzc1, tzc2, tcx, tcy):
    """su, sv, sw on interior cells (nx, ny, nz) from storage tensors."""
    nx, ny, nz = (n - 2 * H for n in u.shape)

    def at(f, di, dj, dk):
        return f[H + di:H + di + nx, H + dj:H + dj + ny, H + dk:H + dk + nz]

    t1 = tzc1.view(1, 1, nz)
    t2 = tzc2.view(1, 1, nz)
    k = torch.arange(nz).view(1, 1, nz)
    below_top = (k < nz - 1).to(u.dtype)
    live = (k >= 1).to(u.dtype)
    sw_live = ((k >= 1) & (k <= nz - 2)).to(u.dtype)
    su = tcx * (at(u, -1, 0, 0) * (at(u, 0, 0, 0) + at(u, -1, 0, 0)) - at(u, 1, 0, 0) * (at(u, 0, 0, 0) + at(u, 1, 0, 0)))
    su = su + tcy * (at(u, 0, -1, 0) * (at(v, 0, -1, 0) + at(v, 1, -1, 0)) - at(u, 0, 1, 0) * (at(v, 0, 0, 0) + at(v, 1, 0, 0)))
    su = su + t1 * at(u, 0, 0, -1) * (at(w, 0, 0, -1) + at(w, 1, 0, -1)) \
        - below_top * t2 * at(u, 0, 0, 1) * (at(w, 0, 0, 0) + at(w, 1, 0, 0))
    sv = tcx * (at(v, -1, 0, 0) * (at(u, -1, 0, 0) + at(u, -1, 1, 0)) - at(v, 1, 0, 0) * (at(u, 0, 0, 0) + at(u, 0, 1, 0)))
    sv = sv + tcy * (at(v, 0, -1, 0) * (at(v, 0, 0, 0) + at(v, 0, -1, 0)) - at(v, 0, 1, 0) * (at(v, 0, 0, 0) + at(v, 0, 1, 0)))
    sv = sv + t1 * at(v, 0, 0, -1) * (at(w, 0, 0, -1) + at(w, 0, 1, -1)) \
        - below_top * t2 * at(v, 0, 0, 1) * (at(w, 0, 0, 0) + at(w, 0, 1, 0))
    sw = tcx * (at(w, -1, 0, 0) * (at(u, -1, 0, 0) + at(u, -1, 0, 1)) - at(w, 1, 0, 0) * (at(u, 0, 0, 0) + at(u, 0, 0, 1)))
    sw = sw + tcy * (at(w, 0, -1, 0) * (at(v, 0, -1, 0) + at(v, 0, -1, 1)) - at(w, 0, 1, 0) * (at(v, 0, 0, 0) + at(v, 0, 0, 1)))
    sw = sw + t1 * at(w, 0, 0, -1) * (at(w, 0, 0, 0) + at(w, 0, 0, -1)) - t2 * at(w, 0, 0, 1) * (at(w, 0, 0, 0) + at(w, 0, 0, 1))
    return su * live, sv * live, sw * sw_live


def test_autograd_adjoint_matches_oracle(oracle):
    for (nx, ny, nz), seed in (((5, 4, 6), 31), ((3, 7, 3), 32), ((1, 2, 4), 33)):
        tzc1, tzc2, tcx, tcy = inputs.coefficients(nz)
        fields = [torch.tensor(a, requires_grad=True) for a in inputs.winds(seed, nx, ny, nz)]
        lams = inputs.normal_fields(seed + 1, nx, ny, nz)
        s = _fwd_torch(*(_pad(f) for f in fields), torch.tensor(tzc1), torch.tensor(tzc2), tcx, tcy)
        loss = sum((torch.tensor(l) * sq).sum() for l, sq in zip(lams, s))
        grads = torch.autograd.grad(loss, fields)
        st = [oracle.pad_periodic(f.detach().numpy(), H) for f in fields]
        sl = [oracle.pad_periodic(l, H) for l in lams]
        ref_s = oracle.fwd(*st, tzc1, tzc2, tcx, tcy, H)
        ref_g = oracle.adj(*st, *sl, tzc1, tzc2, tcx, tcy, H)
        for a, r in zip(s, ref_s):
            r = oracle.interior(r, H)
            assert np.max(np.abs(a.detach().numpy() - r)) <= 1e-14 * max(np.max(np.abs(r)), 1.0)
        for g, r in zip(grads, ref_g):
            r = oracle.interior(r, H)
            assert np.max(np.abs(g.numpy() - r)) <= 1e-13 * max(np.max(np.abs(r)), 1.0), (nx, ny, nz)
