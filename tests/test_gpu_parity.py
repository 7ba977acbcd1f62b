"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Tolerances (stated here and in the design notes):
  * FP64 forward: normwise max |gpu - oracle| / max |oracle| <= 1e-12 per
    output field.  The forward kernels evaluate the same expression tree as
    the oracle without contraction, so the result is also required to be
    bitwise identical.
  * FP64 adjoint: <= 1e-12 normwise (the gather sums the same products in a
    different order than the oracle's scatter).
  * FP32: every cell within 16 * 2^-24 * T(c) + 1e-30, where T(c) is the sum
    of |coef| |A| (|B| + |C|) over the cell's terms (the oracle's error
    magnitude): each term is rounded at most four times and the sum of up to
    six terms at most six times, so 10 units of 2^-24 bound the arithmetic and
    the margin covers the rounding of tzc and tcx to FP32.
"""
import numpy as np
import pytest
import torch

import oracle
from _helpers import H, MARCH_VARIANTS, host_case, log, normwise, oracle_storage

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
SHAPES = [(32, 32, 64, 0), (5, 7, 3, 1), (33, 17, 65, 2), (3, 3, 3, 3), (1, 1, 64, 4), (2, 3, 2, 5),
          (1, 9, 64, 6), (17, 1, 64, 7), (40, 24, 64, 8), (7, 130, 64, 9), (9, 7, 124, 10), (6, 5, 200, 11)]


@pytest.fixture(scope="module")
def pw():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2010_01545_amd import pwadvect
    return pwadvect


def kernels(pw):
    return ["direct", "march"]


def to_dev(arrs, dtype):
    return [torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype) for a in arrs]


def pad_dev(pw, arrs, dtype):
    return [pw.pad_periodic(t, H) for t in to_dev(arrs, dtype)]


def inner(t):
    return t[H:-H, H:-H, H:-H]


def run_fwd(pw, fields, coef, dtype, kernel, sentinel=True):
    tzc1, tzc2, tcx, tcy = coef
    st = pad_dev(pw, fields, dtype)
    outs = [torch.full_like(st[0], float("nan")) if sentinel else torch.zeros_like(st[0]) for _ in range(3)]
    prev = pw.set_kernel(kernel)
    try:
        pw.fwd(*st, torch.from_numpy(tzc1).to(DEV), torch.from_numpy(tzc2).to(DEV), tcx, tcy, H, *outs)
    finally:
        pw.set_kernel(prev)
    torch.cuda.synchronize()
    return [o.cpu().double().numpy() for o in outs]


@pytest.mark.parametrize("kernel", ["direct", "march"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s[:3])))
def test_fwd_f64_matches_oracle(pw, shape, kernel):
    nx, ny, nz, seed = shape
    log("fwd f64 %s %s" % (kernel, shape))
    fields, _, coef = host_case(nx, ny, nz, seed)
    ref = oracle.fwd(*oracle_storage(fields), *coef, H)
    got = run_fwd(pw, fields, coef, torch.float64, kernel)
    for name, g, r in zip(("su", "sv", "sw"), got, ref):
        gi, ri = oracle.interior(g, H), oracle.interior(r, H)
        assert normwise(gi, ri) <= 1e-12, name
        assert np.array_equal(gi, ri), "%s: %d of %d cells differ" % (name, np.sum(gi != ri), gi.size)
        # z-halo levels of interior columns are written with 0
        col = g[H:-H, H:-H, :]
        assert np.all(col[:, :, :H] == 0) and np.all(col[:, :, -H:] == 0), name
        # x/y halo columns are never written
        assert np.all(np.isnan(g[:H])) and np.all(np.isnan(g[-H:])), name
        assert np.all(np.isnan(g[:, :H])) and np.all(np.isnan(g[:, -H:])), name


@pytest.mark.parametrize("kernel", ["direct", "march"])
@pytest.mark.parametrize("shape", SHAPES[:6], ids=lambda s: "x".join(map(str, s[:3])))
def test_fwd_f32_error_bound(pw, shape, kernel):
    nx, ny, nz, seed = shape
    log("fwd f32 %s %s" % (kernel, shape))
    fields, _, coef = host_case(nx, ny, nz, seed)
    f32 = [f.astype(np.float32).astype(np.float64) for f in fields]
    st = oracle_storage(f32)
    ref = oracle.fwd(*st, *coef, H)
    mag = oracle.fwd(*st, *coef, H, abs_bound=True)
    got = run_fwd(pw, f32, coef, torch.float32, kernel)
    for name, g, r, t in zip(("su", "sv", "sw"), got, ref, mag):
        gi, ri, ti = (oracle.interior(a, H) for a in (g, r, t))
        bound = 16 * 2.0 ** -24 * ti + 1e-30
        bad = np.abs(gi - ri) > bound
        assert not np.any(bad), "%s: %d cells exceed the FP32 bound" % (name, np.sum(bad))


def run_adj(pw, fields, lams, coef, dtype, kernel, fused=False):
    tzc1, tzc2, tcx, tcy = coef
    st = pad_dev(pw, fields, dtype)
    sl = pad_dev(pw, lams, dtype)
    t1, t2 = torch.from_numpy(tzc1).to(DEV), torch.from_numpy(tzc2).to(DEV)
    prev = pw.set_kernel(kernel)
    try:
        if fused:
            out = pw.fwd_adj(*st, *sl, t1, t2, tcx, tcy, H)
        else:
            out = pw.adj(*st, *sl, t1, t2, tcx, tcy, H)
    finally:
        pw.set_kernel(prev)
    torch.cuda.synchronize()
    return [o.cpu().double().numpy() for o in out]


@pytest.mark.parametrize("kernel", ["direct", "march"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s[:3])))
def test_adj_f64_matches_oracle(pw, shape, kernel):
    nx, ny, nz, seed = shape
    log("adj f64 %s %s" % (kernel, shape))
    fields, lams, coef = host_case(nx, ny, nz, seed, lam_seed=seed + 50)
    ref = oracle.adj(*oracle_storage(fields), *oracle_storage(lams), *coef, H)
    got = run_adj(pw, fields, lams, coef, torch.float64, kernel)
    for name, g, r in zip(("gu", "gv", "gw"), got, ref):
        assert normwise(oracle.interior(g, H), oracle.interior(r, H)) <= 1e-12, name


@pytest.mark.parametrize("kernel", ["direct", "march"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s[:3])))
def test_adj_f32_error_bound(pw, shape, kernel):
    """FP32 gather adjoint against the FP64 oracle on the same FP32-rounded
    inputs: each gradient entry sums up to 22 rounded products of three
    factors, so 32 units of 2^-24 times the sum of their absolute values
    bound the FP32 arithmetic."""
    nx, ny, nz, seed = shape
    log("adj f32 %s %s" % (kernel, shape))
    fields, lams, coef = host_case(nx, ny, nz, seed, lam_seed=seed + 70)
    f32 = [a.astype(np.float32).astype(np.float64) for a in fields]
    l32 = [a.astype(np.float32).astype(np.float64) for a in lams]
    st, sl = oracle_storage(f32), oracle_storage(l32)
    ref = oracle.adj(*st, *sl, *coef, H)
    mag = oracle.adj(*st, *sl, *coef, H, abs_bound=True)
    got = run_adj(pw, f32, l32, coef, torch.float32, kernel)
    for name, g, r, t in zip(("gu", "gv", "gw"), got, ref, mag):
        gi, ri, ti = (oracle.interior(a, H) for a in (g, r, t))
        bad = np.abs(gi - ri) > 32 * 2.0 ** -24 * ti + 1e-30
        assert not np.any(bad), "%s: %d cells exceed the FP32 bound" % (name, np.sum(bad))


@pytest.mark.parametrize("kernel", ["direct", "march"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_fused_equals_separate(pw, kernel, dtype):
    nx, ny, nz, seed = 40, 24, 64, 11
    log("fused %s %s" % (kernel, dtype))
    fields, lams, coef = host_case(nx, ny, nz, seed, lam_seed=seed + 50)
    s = run_fwd(pw, fields, coef, dtype, kernel, sentinel=False)
    g = run_adj(pw, fields, lams, coef, dtype, kernel)
    f = run_adj(pw, fields, lams, coef, dtype, kernel, fused=True)
    for a, b in zip(s + g, f):
        assert np.array_equal(oracle.interior(a, H), oracle.interior(b, H))


@pytest.mark.parametrize("kernel", ["direct", "march"])
def test_deterministic(pw, kernel):
    fields, lams, coef = host_case(33, 20, 64, 12, lam_seed=62)
    a = run_adj(pw, fields, lams, coef, torch.float64, kernel, fused=True)
    b = run_adj(pw, fields, lams, coef, torch.float64, kernel, fused=True)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_march_and_direct_agree_bitwise(pw, dtype):
    """Both kernel families evaluate the same per-cell trees without
    contraction, so they agree bit for bit (forward and adjoint)."""
    fields, lams, coef = host_case(64, 48, 64, 13, lam_seed=63)
    a = run_adj(pw, fields, lams, coef, dtype, "direct", fused=True)
    b = run_adj(pw, fields, lams, coef, dtype, "march", fused=True)
    for x, y in zip(a, b):
        assert np.array_equal(oracle.interior(x, H), oracle.interior(y, H))


@pytest.mark.parametrize("order", ["xcd", "natural", 3])
@pytest.mark.parametrize("shape", [(45, 31, 64, 14), (12, 17, 40, 16)], ids=lambda s: "x".join(map(str, s[:3])))
@pytest.mark.parametrize("variant", MARCH_VARIANTS)
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_every_march_variant_matches_direct(pw, variant, dtype, shape, order):
    """Each strip-width / prefetch-depth / halo-carrier variant of the
    x-marching kernel, in three block orders (XCD ranges, natural, groups of
    3 strips per XCD) and with a short march length (so
    several x-segments meet), gives the direct kernel's bits, forward, adjoint
    and fused.  ny = 31 and 17 leave last strips one column and several
    columns narrower than every strip width, and a one-column strip."""
    nx, ny, nz, seed = shape
    log("variant %s %s %s %s" % (variant, dtype, shape, order))
    fields, lams, coef = host_case(nx, ny, nz, seed, lam_seed=seed + 50)
    ref_f = run_fwd(pw, fields, coef, dtype, "direct", sentinel=False)
    ref_a = run_adj(pw, fields, lams, coef, dtype, "direct", fused=True)
    with pw.tuning(variant=variant, lx=7, order=order):
        got_f = run_fwd(pw, fields, coef, dtype, "march", sentinel=False)
        got_a = run_adj(pw, fields, lams, coef, dtype, "march", fused=True)
        got_g = run_adj(pw, fields, lams, coef, dtype, "march", fused=False)
    for x, y in zip(ref_f + ref_a, got_f + got_a):
        assert np.array_equal(oracle.interior(x, H), oracle.interior(y, H))
    for x, y in zip(ref_a[3:], got_g):
        assert np.array_equal(oracle.interior(x, H), oracle.interior(y, H))


@pytest.mark.parametrize("kernel", ["direct", "march"])
@pytest.mark.parametrize("halo", [1, 3, 5])
@pytest.mark.parametrize("shape", [(9, 10, 64, 21), (5, 4, 7, 22)], ids=lambda s: "x".join(map(str, s[:3])))
def test_other_halo_widths(pw, kernel, halo, shape):
    """Storage with halo 1, 3 and 5 (the scheme reads only the first halo
    layer; the rest is layout): forward bitwise, adjoint within 1e-12."""
    nx, ny, nz, seed = shape
    log("halo %d %s %s" % (halo, kernel, shape))
    fields, lams, coef = host_case(nx, ny, nz, seed, lam_seed=seed + 5)
    tzc1, tzc2, tcx, tcy = coef
    st_h = [oracle.pad_periodic(a, halo) for a in fields]
    sl_h = [oracle.pad_periodic(a, halo) for a in lams]
    ref_s = oracle.fwd(*st_h, *coef, halo)
    ref_g = oracle.adj(*st_h, *sl_h, *coef, halo)
    st = [pw.pad_periodic(t, halo) for t in to_dev(fields, torch.float64)]
    sl = [pw.pad_periodic(t, halo) for t in to_dev(lams, torch.float64)]
    t1, t2 = torch.from_numpy(tzc1).to(DEV), torch.from_numpy(tzc2).to(DEV)
    prev = pw.set_kernel(kernel)
    try:
        out = pw.fwd_adj(*st, *sl, t1, t2, tcx, tcy, halo)
    finally:
        pw.set_kernel(prev)
    torch.cuda.synchronize()
    inner_h = lambda a: a[halo:-halo, halo:-halo, halo:-halo]
    for got, ref in zip(out[:3], ref_s):
        assert np.array_equal(inner_h(got.cpu().numpy()), inner_h(ref))
    for got, ref in zip(out[3:], ref_g):
        assert normwise(inner_h(got.cpu().numpy()), inner_h(ref)) <= 1e-12


def test_march_selection_limits(pw):
    """The x-marching kernel takes halos of at most 32 levels; asked for a
    wider one it is refused before any launch, and "auto" falls back to the
    direct kernel."""
    halo = 33
    fields, _, coef = host_case(4, 3, 8, 90)
    st = [pw.pad_periodic(t, halo) for t in to_dev(fields, torch.float64)]
    t1, t2 = torch.from_numpy(coef[0]).to(DEV), torch.from_numpy(coef[1]).to(DEV)
    prev = pw.set_kernel("march")
    try:
        with pytest.raises(pw.PWError) as e:
            pw.fwd(*st, t1, t2, coef[2], coef[3], halo)
        assert e.value.code == -5
    finally:
        pw.set_kernel(prev)
    got = pw.fwd(*st, t1, t2, coef[2], coef[3], halo)
    torch.cuda.synchronize()
    ref = oracle.fwd(*[oracle.pad_periodic(a, halo) for a in fields], *coef, halo)
    for g, r in zip(got, ref):
        gi = g.cpu().numpy()[halo:-halo, halo:-halo, halo:-halo]
        assert np.array_equal(gi, r[halo:-halo, halo:-halo, halo:-halo])


@pytest.mark.parametrize("variant", MARCH_VARIANTS)
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_tall_columns_every_variant_matches_direct(pw, variant, dtype):
    """Columns taller than a wavefront are marched in z-chunks of 62 levels
    (chunk halo lanes 0 and 63): every variant, with short x-segments, gives
    the direct kernel's bits for the forward, the adjoint and the fused pass."""
    fields, lams, coef = host_case(13, 11, 150, 15, lam_seed=65)
    ref_f = run_fwd(pw, fields, coef, dtype, "direct", sentinel=False)
    ref_a = run_adj(pw, fields, lams, coef, dtype, "direct", fused=True)
    with pw.tuning(variant=variant, lx=4):
        got_f = run_fwd(pw, fields, coef, dtype, "march", sentinel=True)
        got_a = run_adj(pw, fields, lams, coef, dtype, "march", fused=True)
    for x, y in zip(ref_f + ref_a, got_f + got_a):
        assert np.array_equal(oracle.interior(x, H), oracle.interior(y, H))
    for g in got_f:   # every interior column fully written, halo columns untouched
        col = g[H:-H, H:-H, :]
        assert not np.any(np.isnan(col))
        assert np.all(col[:, :, :H] == 0) and np.all(col[:, :, -H:] == 0)
        assert np.all(np.isnan(g[:H])) and np.all(np.isnan(g[:, :H]))


@pytest.mark.parametrize("variant", [5, 6])
@pytest.mark.parametrize("halo", [1, 3])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_edge_wave_variants_other_halos(pw, variant, halo, dtype):
    """The edge-wave variants address their extra halo column through the
    storage geometry: with halo 1 and 3 (and a last strip one column and
    several columns short of the strip width) the fused pass gives the direct
    kernel's bits."""
    log("edge-wave variant %s halo %d %s" % (variant, halo, dtype))
    fields, lams, coef = host_case(11, 23, 40, 17, lam_seed=67)
    tzc1, tzc2, tcx, tcy = coef
    st = [pw.pad_periodic(t, halo) for t in to_dev(fields, dtype)]
    sl = [pw.pad_periodic(t, halo) for t in to_dev(lams, dtype)]
    t1, t2 = torch.from_numpy(tzc1).to(DEV), torch.from_numpy(tzc2).to(DEV)
    res = {}
    for kernel in ("direct", "march"):
        with pw.tuning(kernel=kernel, variant=variant, lx=5):
            res[kernel] = [o.cpu().numpy() for o in pw.fwd_adj(*st, *sl, t1, t2, tcx, tcy, halo)]
    inner_h = lambda a: a[halo:-halo, halo:-halo, halo:-halo]
    for a, b in zip(res["direct"], res["march"]):
        assert np.array_equal(inner_h(a), inner_h(b))
