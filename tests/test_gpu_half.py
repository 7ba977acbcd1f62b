"""GPU parity of the 16-bit storage dtypes (PW_F16: IEEE binary16, PW_BF16:
bfloat16), both computed in float.

The oracle runs in FP64 on the same 16-bit inputs (widened exactly).  Bounds,
with u16 the storage type's unit roundoff (2^-11 for binary16, 2^-8 for
bfloat16) and T the oracle's error magnitude of the cell (sum of absolute
products):
  * forward: 16 * 2^-24 * T (the FP32 bound of the float arithmetic) plus one
    rounding of the result to 16 bits, u16 * |ref|, plus 2^-25 for binary16
    results in the subnormal range;
  * adjoint: 32 * 2^-24 * T plus the same result rounding.
Kernel families, marching variants and fused and separate launches must agree
bit for bit, as for the wider types.  The offload of 16-bit host arrays is
checked against the oracle in test_gpu_offload.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2010_01545_amd import inputs
from _helpers import H, MARCH_VARIANTS, host_case, log, oracle_storage

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
TYPES = {"f16": (torch.float16, 2.0 ** -11, 2.0 ** -25), "bf16": (torch.bfloat16, 2.0 ** -8, 0.0)}
SHAPES = [(32, 32, 64, 80), (33, 17, 65, 81), (5, 7, 3, 82), (7, 130, 64, 83), (1, 9, 64, 84)]


@pytest.fixture(scope="module")
def pw():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2010_01545_amd import pwadvect
    return pwadvect


def rounded(arrs, kind):
    return [inputs.round_storage(a, kind) for a in arrs]


def dev(arrs, dtype):
    return [torch.from_numpy(oracle.pad_periodic(a, H)).to(DEV, dtype) for a in arrs]


def coef_dev(coef):
    return torch.from_numpy(coef[0]).to(DEV), torch.from_numpy(coef[1]).to(DEV), coef[2], coef[3]


def host(ts):
    return [t.cpu().double().numpy() for t in ts]


def with_kernel(pw, kernel, fn):
    prev = pw.set_kernel(kernel)
    try:
        out = fn()
    finally:
        pw.set_kernel(prev)
    torch.cuda.synchronize()
    return host(out)


@pytest.mark.parametrize("kernel", ["direct", "march"])
@pytest.mark.parametrize("kind", list(TYPES))
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s[:3])))
def test_fwd_and_adj_bounds(pw, shape, kind, kernel):
    nx, ny, nz, seed = shape
    dtype, u16, sub = TYPES[kind]
    log("%s fwd/adj %s %s" % (kind, kernel, shape))
    fields, lams, coef = host_case(nx, ny, nz, seed, lam_seed=seed + 1)
    f16, l16 = rounded(fields, kind), rounded(lams, kind)
    st, sl = oracle_storage(f16), oracle_storage(l16)
    st_d, sl_d = dev(f16, dtype), dev(l16, dtype)
    outs = [torch.full_like(st_d[0], float("nan")) for _ in range(3)]
    got_s = with_kernel(pw, kernel, lambda: pw.fwd(*st_d, *coef_dev(coef), H, *outs))
    got_g = with_kernel(pw, kernel, lambda: pw.adj(*st_d, *sl_d, *coef_dev(coef), H))
    ref_s, mag_s = oracle.fwd(*st, *coef, H), oracle.fwd(*st, *coef, H, abs_bound=True)
    ref_g, mag_g = oracle.adj(*st, *sl, *coef, H), oracle.adj(*st, *sl, *coef, H, abs_bound=True)
    for name, got, ref, mag, units in (("fwd", got_s, ref_s, mag_s, 16), ("adj", got_g, ref_g, mag_g, 32)):
        for q in range(3):
            g, r, t = (oracle.interior(a, H) for a in (got[q], ref[q], mag[q]))
            bound = units * 2.0 ** -24 * t + u16 * np.abs(r) + sub + 1e-30
            bad = np.abs(g - r) > bound
            assert not np.any(bad), "%s %d: %d cells exceed the bound" % (name, q, np.sum(bad))
    for o in got_s:   # layout: zero z halo, untouched x/y halo columns
        col = o[H:-H, H:-H, :]
        assert np.all(col[:, :, :H] == 0) and np.all(col[:, :, -H:] == 0)
        assert np.all(np.isnan(o[:H])) and np.all(np.isnan(o[:, :H]))


@pytest.mark.parametrize("kind", list(TYPES))
def test_fused_separate_and_kernels_agree(pw, kind):
    dtype = TYPES[kind][0]
    fields, lams, coef = host_case(45, 31, 64, 85, lam_seed=86)
    st, sl = dev(rounded(fields, kind), dtype), dev(rounded(lams, kind), dtype)
    c = coef_dev(coef)
    results = {}
    for kernel in ("direct", "march"):
        s = with_kernel(pw, kernel, lambda: pw.fwd(*st, *c, H))
        g = with_kernel(pw, kernel, lambda: pw.adj(*st, *sl, *c, H))
        f = with_kernel(pw, kernel, lambda: pw.fwd_adj(*st, *sl, *c, H))
        for a, b in zip(s + g, f):
            assert np.array_equal(oracle.interior(a, H), oracle.interior(b, H))
        results[kernel] = f
    for a, b in zip(results["direct"], results["march"]):
        assert np.array_equal(oracle.interior(a, H), oracle.interior(b, H))
    for v in MARCH_VARIANTS:
        for order in ("xcd", "natural"):
            with pw.tuning(variant=v, lx=7, order=order):
                f = with_kernel(pw, "march", lambda: pw.fwd_adj(*st, *sl, *c, H))
            for a, b in zip(results["direct"], f):
                assert np.array_equal(oracle.interior(a, H), oracle.interior(b, H)), (v, order)


@pytest.mark.parametrize("kind", list(TYPES))
def test_update(pw, kind):
    dtype, u16, sub = TYPES[kind]
    fields, base, coef = host_case(20, 13, 64, 87, lam_seed=88)
    f16, b16 = rounded(fields, kind), rounded(base, kind)
    st, sb = dev(f16, dtype), dev(b16, dtype)
    c = coef_dev(coef)
    beta = 0.8125
    got = host(pw.fwd_update(*st, *c, H, *sb, beta))
    ref = oracle.fwd_update(*oracle_storage(f16), *coef, H, *oracle_storage(b16), beta)
    mag = oracle.fwd(*oracle_storage(f16), *coef, H, abs_bound=True)
    for q in range(3):
        g, r, t = (oracle.interior(a, H) for a in (got[q], ref[q], mag[q]))
        bound = 2.0 ** -24 * (16 * beta * t + 2 * (np.abs(r) + beta * t)) + u16 * np.abs(r) + sub + 1e-30
        assert not np.any(np.abs(g - r) > bound), q
