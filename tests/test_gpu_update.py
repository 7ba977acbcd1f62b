"""GPU parity of the update form pw_advect_fwd_update, o = b + beta * s.

The forward is bitwise equal to the oracle in FP64 and the update is the same
two rounded operations on both sides, so FP64 results must equal the oracle
bit for bit in every mode: in-place accumulation (b = o), the fused Euler
step (b = u, v, w) and separate base arrays.  FP32-storage/FP64-arithmetic
results must equal the oracle's FP64 result rounded to float.  FP32 results
are bounded by the forward's FP32 bound scaled by |beta| plus two roundings
of the result.
"""

import numpy as np
import pytest
import torch

import oracle
from _helpers import H, MARCH_VARIANTS, host_case, log, oracle_storage

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
SHAPES = [(32, 32, 64, 60), (33, 17, 65, 61), (5, 7, 3, 62), (7, 130, 64, 63), (1, 1, 64, 64)]
MODES = ["in_place", "euler", "separate"]


@pytest.fixture(scope="module")
def pw():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2010_01545_amd import pwadvect
    return pwadvect


def dev(arrs, dtype):
    return [torch.from_numpy(oracle.pad_periodic(a, H)).to(DEV, dtype) for a in arrs]


def run(pw, kernel, mode, fields, base, coef, beta, dtype, compute=None):
    """Returns (o arrays on the host, the b arrays the call used, as float64)."""
    tzc1, tzc2, tcx, tcy = coef
    st = dev(fields, dtype)
    t1, t2 = torch.from_numpy(tzc1).to(DEV), torch.from_numpy(tzc2).to(DEV)
    if mode == "euler":
        b = st
        o = [torch.full_like(st[0], float("nan")) for _ in range(3)]
    elif mode == "in_place":
        o = dev(base, dtype)
        for t in o:  # x/y halo columns of o must survive: mark them
            t[:H] = float("nan"); t[-H:] = float("nan"); t[:, :H] = float("nan"); t[:, -H:] = float("nan")
        b = o
    else:
        b = dev(base, dtype)
        o = [torch.full_like(st[0], float("nan")) for _ in range(3)]
    b_host = [t.cpu().double().numpy().copy() for t in b]
    prev = pw.set_kernel(kernel)
    try:
        pw.fwd_update(*st, t1, t2, tcx, tcy, H, *b, beta, *o, compute=compute)
    finally:
        pw.set_kernel(prev)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in o], b_host


def check_layout(o):
    for g in o:
        col = g[H:-H, H:-H, :]
        assert np.all(col[:, :, :H] == 0) and np.all(col[:, :, -H:] == 0)
        assert np.all(np.isnan(g[:H])) and np.all(np.isnan(g[-H:]))
        assert np.all(np.isnan(g[:, :H])) and np.all(np.isnan(g[:, -H:]))


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("kernel", ["direct", "march"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s[:3])))
def test_update_f64_bitwise(pw, shape, kernel, mode):
    nx, ny, nz, seed = shape
    log("update f64 %s %s %s" % (kernel, mode, shape))
    fields, base, coef = host_case(nx, ny, nz, seed, lam_seed=seed + 3)
    beta = 0.37 if mode != "in_place" else 1.0
    o, b = run(pw, kernel, mode, fields, base, coef, beta, torch.float64)
    ref = oracle.fwd_update(*oracle_storage(fields), *coef, H, *b, beta)
    for q in range(3):
        gi, ri = oracle.interior(o[q], H), oracle.interior(ref[q], H)
        assert np.array_equal(gi, ri), "%d: %d of %d cells differ" % (q, np.sum(gi != ri), gi.size)
    check_layout(o)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("kernel", ["direct", "march"])
def test_update_mixed_is_rounded_oracle(pw, kernel, mode):
    nx, ny, nz, seed = 24, 20, 64, 65
    log("update f32/f64 %s %s" % (kernel, mode))
    fields, base, coef = host_case(nx, ny, nz, seed, lam_seed=seed + 3)
    f32 = [a.astype(np.float32).astype(np.float64) for a in fields]
    b32 = [a.astype(np.float32).astype(np.float64) for a in base]
    beta = -0.61
    o, b = run(pw, kernel, mode, f32, b32, coef, beta, torch.float32, compute=torch.float64)
    ref = oracle.fwd_update(*oracle_storage(f32), *coef, H, *b, beta)
    for q in range(3):
        gi, ri = oracle.interior(o[q], H), oracle.interior(ref[q], H).astype(np.float32)
        assert np.array_equal(gi, ri), "%d: %d cells differ" % (q, np.sum(gi != ri))
    check_layout(o)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("kernel", ["direct", "march"])
def test_update_f32_bound(pw, kernel, mode):
    nx, ny, nz, seed = 24, 20, 64, 66
    log("update f32 %s %s" % (kernel, mode))
    fields, base, coef = host_case(nx, ny, nz, seed, lam_seed=seed + 3)
    f32 = [a.astype(np.float32).astype(np.float64) for a in fields]
    b32 = [a.astype(np.float32).astype(np.float64) for a in base]
    beta = 0.8125   # exact in FP32
    o, b = run(pw, kernel, mode, f32, b32, coef, beta, torch.float32)
    st = oracle_storage(f32)
    ref = oracle.fwd_update(*st, *coef, H, *b, beta)
    mag = oracle.fwd(*st, *coef, H, abs_bound=True)
    for q in range(3):
        gi = oracle.interior(o[q], H).astype(np.float64)
        ri, ti = oracle.interior(ref[q], H), oracle.interior(mag[q], H)
        # FP32 forward error (16 units of T) times |beta|, then the rounding of
        # beta * s and of the sum (each at most one unit of the result's size)
        bound = 2.0 ** -24 * (16 * abs(beta) * ti + 2 * (np.abs(ri) + abs(beta) * ti)) + 1e-30
        bad = np.abs(gi - ri) > bound
        assert not np.any(bad), "%d: %d cells exceed the FP32 bound" % (q, np.sum(bad))
    check_layout(o)


@pytest.mark.parametrize("order", ["xcd", "natural"])
@pytest.mark.parametrize("variant", MARCH_VARIANTS)
@pytest.mark.parametrize("mode", MODES)
def test_update_march_variants_match_direct(pw, variant, mode, order):
    fields, base, coef = host_case(45, 31, 64, 67, lam_seed=68)
    ref, _ = run(pw, "direct", mode, fields, base, coef, 0.29, torch.float64)
    with pw.tuning(variant=variant, lx=7, order=order):
        got, _ = run(pw, "march", mode, fields, base, coef, 0.29, torch.float64)
    for x, y in zip(ref, got):
        assert np.array_equal(oracle.interior(x, H), oracle.interior(y, H))


def test_update_equals_forward_then_axpy(pw):
    """The fused Euler step gives the bits of the forward followed by the same
    two operations done separately with torch (u + dt * su, unfused)."""
    fields, _, coef = host_case(40, 24, 64, 69)
    tzc1, tzc2, tcx, tcy = coef
    st = dev(fields, torch.float64)
    t1, t2 = torch.from_numpy(tzc1).to(DEV), torch.from_numpy(tzc2).to(DEV)
    s = pw.fwd(*st, t1, t2, tcx, tcy, H)
    dt = 0.125 * 3
    o = pw.fwd_update(*st, t1, t2, tcx, tcy, H, *st, dt)
    for f, sf, of in zip(st, s, o):
        sep = f + torch.mul(sf, dt)
        assert torch.equal(of[H:-H, H:-H, H:-H], sep[H:-H, H:-H, H:-H])
