"""GPU tests of the x-marching kernels for columns of more than 64 levels,
held by two to four wavefronts of one workgroup (in z-chunks above 256
levels) whose z-neighbours come from the LDS ring: bit for bit against the
direct kernel (which is tested against the oracle in test_gpu_parity),
forward, adjoint, fused pass and both update forms, for every storage type,
at heights on both sides of 128, 192 and 256 and in chunks of each
wavefront count, with several x-segments, narrow last strips, three block
orders and halo widths 1 to 3; and once against the oracle itself."""
import numpy as np
import pytest
import torch

import oracle
from paper_2010_01545_amd import inputs
from _helpers import host_case, log, oracle_storage

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")

KINDS = {"f64": (torch.float64, None), "f32": (torch.float32, None), "f32f64": (torch.float32, torch.float64),
         "f16": (torch.float16, None), "bf16": (torch.bfloat16, None)}


@pytest.fixture(scope="module")
def pw():
    assert torch.cuda.is_available()
    from paper_2010_01545_amd import pwadvect
    return pwadvect


def _stage(pw, arrs, dtype, h):
    return [pw.pad_periodic(torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype), h) for a in arrs]


def _run(pw, fields, lams, coef, dtype, compute, h, path, kernel, tune):
    """One call of `path` with the given kernel family and tuning; returns
    every output as float64 numpy storage arrays (NaN where not written)."""
    tzc1, tzc2, tcx, tcy = coef
    st = _stage(pw, fields, dtype, h)
    t1, t2 = torch.from_numpy(tzc1).to(DEV), torch.from_numpy(tzc2).to(DEV)
    nan = lambda: torch.full_like(st[0], float("nan"))
    with pw.tuning(kernel=kernel, **tune):
        if path == "fwd":
            out = pw.fwd(*st, t1, t2, tcx, tcy, h, nan(), nan(), nan(), compute=compute)
        elif path == "euler":
            out = pw.fwd_update(*st, t1, t2, tcx, tcy, h, *st, 0.25, nan(), nan(), nan(), compute=compute)
        elif path == "accumulate":
            base = _stage(pw, lams, dtype, h)
            out = pw.fwd_update(*st, t1, t2, tcx, tcy, h, *base, -0.5, *base, compute=compute)
        else:
            sl = _stage(pw, lams, dtype, h)
            if path == "adj":
                out = pw.adj(*st, *sl, t1, t2, tcx, tcy, h, nan(), nan(), nan(), compute=compute)
            else:
                out = pw.fwd_adj(*st, *sl, t1, t2, tcx, tcy, h, out=[nan() for _ in range(6)], compute=compute)
    torch.cuda.synchronize()
    return [o.cpu().double().numpy() for o in out]


def _same(a, b):
    """Equal bits where written, and unwritten (NaN) at the same places."""
    return np.array_equal(np.isnan(a), np.isnan(b)) and np.array_equal(np.nan_to_num(a), np.nan_to_num(b))


@pytest.mark.parametrize("nz", [65, 100, 128, 129, 150, 192, 193, 256, 257, 400, 508, 509])
@pytest.mark.parametrize("kind", list(KINDS))
def test_tall_columns_match_direct(pw, kind, nz):
    """Default kernel selection (two wavefronts per column up to 128 levels,
    three up to 192, four up to 256; above that z-chunks of 126, 190 or 254
    levels: 257 levels in two chunks of three wavefronts, 400 and 508 in two
    of four, 509 in three of three) against the direct kernel, with
    x-segments of 5 planes and ny = 11, which leaves a last strip narrower
    than the strip width."""
    dtype, compute = KINDS[kind]
    nx, ny, h, seed = 13, 11, 2, 300 + nz
    log("tall %s nz=%d" % (kind, nz))
    fields, lams, coef = host_case(nx, ny, nz, seed, lam_seed=seed + 1)
    for path in ("fwd", "adj", "fused", "euler", "accumulate"):
        ref = _run(pw, fields, lams, coef, dtype, compute, h, path, "direct", {})
        got = _run(pw, fields, lams, coef, dtype, compute, h, path, "march", dict(lx=5))
        for q, (a, b) in enumerate(zip(ref, got)):
            assert _same(a, b), (path, q)


@pytest.mark.parametrize("order", ["xcd", "natural", 2])
@pytest.mark.parametrize("shape", [(9, 7, 100, 1), (6, 5, 256, 1), (7, 9, 150, 3), (5, 3, 70, 3), (6, 11, 180, 2),
                                   (5, 6, 300, 3)],
                         ids=lambda s: "x".join(map(str, s[:3])) + "h%d" % s[3])
def test_tall_orders_and_halos(pw, shape, order):
    """Block orders and halo widths 1 and 3 (the edge waves address their
    halo column through the storage geometry), FP64 forward and fused pass."""
    nx, ny, nz, h = shape
    log("tall order %s shape %s" % (order, shape))
    fields, lams, coef = host_case(nx, ny, nz, 400 + nz, lam_seed=401 + nz)
    for path in ("fwd", "fused"):
        ref = _run(pw, fields, lams, coef, torch.float64, None, h, path, "direct", {})
        for lx in (0, 3):
            got = _run(pw, fields, lams, coef, torch.float64, None, h, path, "march",
                       dict(lx=lx, order=order, variant=pw.MARCH_VARIANTS - 1))
            for q, (a, b) in enumerate(zip(ref, got)):
                assert _same(a, b), (path, lx, q)


@pytest.mark.parametrize("waves", [2, 3, 4])
@pytest.mark.parametrize("nz", [65, 130, 255, 300, 520])
@pytest.mark.parametrize("kind", ["f64", "f32", "bf16"])
def test_tall_wave_counts(pw, kind, nz, waves):
    """Each count of wavefronts per column, chosen with the tuning knob, at
    heights that one workgroup holds with idle lanes and at heights cut into
    two to five z-chunks (520 levels: five chunks of 126, three of 190, three
    of 254), forward, adjoint and fused pass against the direct kernel."""
    dtype, compute = KINDS[kind]
    nx, ny, h, seed = 7, 9, 2, 500 + nz + waves
    log("tall waves %d %s nz=%d" % (waves, kind, nz))
    fields, lams, coef = host_case(nx, ny, nz, seed, lam_seed=seed + 1)
    for path in ("fwd", "adj", "fused"):
        ref = _run(pw, fields, lams, coef, dtype, compute, h, path, "direct", {})
        got = _run(pw, fields, lams, coef, dtype, compute, h, path, "march", dict(lx=4, tall_waves=waves))
        for q, (a, b) in enumerate(zip(ref, got)):
            assert _same(a, b), (path, q)


@pytest.mark.parametrize("shape", [(5, 4, 1000, 1), (4, 5, 300, 32), (3, 4, 129, 32)],
                         ids=lambda s: "x".join(map(str, s[:3])) + "h%d" % s[3])
@pytest.mark.parametrize("kind", ["f64", "f32"])
def test_tall_extremes(pw, kind, shape):
    """A column of 1000 levels (four z-chunks of four wavefronts) with halo 1,
    and the widest halo the x-marching kernels take (32, whose z-halo pads
    fill a whole wavefront of lanes at each end of a column) at 300 and 129
    levels: forward, adjoint and fused pass against the direct kernel."""
    nx, ny, nz, h = shape
    dtype, compute = KINDS[kind]
    log("tall extreme %s %s" % (kind, shape))
    fields, lams, coef = host_case(nx, ny, nz, 600 + nz + h, lam_seed=601 + nz + h)
    for path in ("fwd", "adj", "fused"):
        ref = _run(pw, fields, lams, coef, dtype, compute, h, path, "direct", {})
        got = _run(pw, fields, lams, coef, dtype, compute, h, path, "march", {})
        for q, (a, b) in enumerate(zip(ref, got)):
            assert _same(a, b), (path, q)


def test_tall_columns_match_oracle(pw):
    """FP64 forward and fused pass at 150 levels against the oracle: bitwise
    forward, adjoint within 1e-12 normwise; every interior column fully
    written (with zero z-halo levels), halo columns untouched."""
    nx, ny, nz, h = 10, 9, 150, inputs.HALO
    fields, lams, coef = host_case(nx, ny, nz, 77, lam_seed=78)
    st, sl = oracle_storage(fields), oracle_storage(lams)
    ref_s = oracle.fwd(*st, *coef, h)
    ref_g = oracle.adj(*st, *sl, *coef, h)
    got = _run(pw, fields, lams, coef, torch.float64, None, h, "fused", "march", {})
    for g, r in zip(got[:3], ref_s):
        assert np.array_equal(oracle.interior(g, h), oracle.interior(r, h))
    for g, r in zip(got[3:], ref_g):
        gi, ri = oracle.interior(g, h), oracle.interior(r, h)
        assert np.max(np.abs(gi - ri)) <= 1e-12 * np.max(np.abs(ri))
    for g in got:
        col = g[h:-h, h:-h, :]
        assert not np.any(np.isnan(col))
        assert np.all(col[:, :, :h] == 0) and np.all(col[:, :, -h:] == 0)
        assert np.all(np.isnan(g[:h])) and np.all(np.isnan(g[:, :h]))
