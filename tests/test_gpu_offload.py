"""GPU tests of the host-resident offload path (pw_advect_fwd_host), against
the oracle.

For every storage type the offload of host arrays must match the FP64 oracle
on the same (storage-rounded) inputs with the bar of the device path for that
type (bitwise for FP64; bitwise to the oracle rounded to float for FP32
storage with FP64 arithmetic; the FP32 and 16-bit error bounds otherwise, see
test_gpu_parity and test_gpu_half), give the device path's bits, write only
interior columns of the host outputs, and order itself on the caller's
stream.  Shapes include odd ny and odd nz with halo 1 and 2, whose 16-bit
output rows are not a multiple of 4 bytes long, for each way the outputs come
back: pinned memory through the runtime's copies, through the library's copy
kernel, written by the advection kernel itself, or by whichever of these the
automatic mode (the default) picks, and pageable memory.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2010_01545_amd import inputs
from _helpers import host_case, log

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")

# storage dtype, arithmetic dtype (None: the storage dtype), inputs.round_storage kind
KINDS = {
    "f64": (torch.float64, None, "f64"),
    "f32": (torch.float32, None, "f32"),
    "f32f64": (torch.float32, torch.float64, "f32"),
    "f16": (torch.float16, None, "f16"),
    "bf16": (torch.bfloat16, None, "bf16"),
}
# (nx, ny, nz, halo, seed), chunk sizes
SHAPES = [((20, 13, 64, 2, 31), (1, 3, 7, 20)),
          ((9, 7, 7, 2, 32), (4, 9)),
          ((5, 7, 3, 2, 35), (2, 5)),
          ((9, 7, 3, 1, 36), (2, 4)),
          ((6, 5, 3, 1, 34), (5,)),
          ((7, 6, 150, 2, 38), (3, 7))]       # columns of 150 levels: the tall-column kernels
MODES = ["pinned_runtime_copy", "pinned_copy_kernel", "pinned_direct", "pinned_auto", "pageable"]
COPY_OUT = {"pinned_runtime_copy": "runtime", "pinned_copy_kernel": "kernel", "pinned_direct": "direct",
            "pinned_auto": "auto", "pageable": "auto"}


@pytest.fixture(scope="module")
def pw():
    assert torch.cuda.is_available()
    from paper_2010_01545_amd import pwadvect
    return pwadvect


def _host(arr, dtype, pinned):
    t = torch.empty(arr.shape, dtype=dtype, pin_memory=pinned)
    t.copy_(torch.from_numpy(arr))      # exact: arr already holds storage-type values
    return t


def within_bar(kind, got, ref, mag):
    """The device path's parity bar for storage kind ``kind``: got and ref
    are interior float64 arrays, mag the oracle's error magnitude T."""
    if kind == "f64":
        return np.array_equal(got, ref)
    if kind == "f32f64":
        return np.array_equal(got, ref.astype(np.float32).astype(np.float64))
    u16, sub = {"f32": (0.0, 0.0), "f16": (2.0 ** -11, 2.0 ** -25), "bf16": (2.0 ** -8, 0.0)}[kind]
    bound = 16 * 2.0 ** -24 * mag + u16 * np.abs(ref) + sub
    return not np.any(np.abs(got - ref) > bound)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("kind", list(KINDS))
@pytest.mark.parametrize("shape,chunks", SHAPES, ids=["x".join(map(str, s[0][:3])) + "h%d" % s[0][3]
                                                       for s in SHAPES])
def test_offload_matches_oracle(pw, shape, chunks, kind, mode):
    nx, ny, nz, h, seed = shape
    dtype, compute, rk = KINDS[kind]
    pinned = mode != "pageable"
    fields, _, coef = host_case(nx, ny, nz, seed)
    tzc1, tzc2, tcx, tcy = coef
    st = [oracle.pad_periodic(inputs.round_storage(f, rk), h) for f in fields]   # host storage, FP64 values
    ref = oracle.fwd(*st, tzc1, tzc2, tcx, tcy, h)
    mag = oracle.fwd(*st, tzc1, tzc2, tcx, tcy, h, abs_bound=True)
    t1, t2 = torch.from_numpy(tzc1).to(DEV), torch.from_numpy(tzc2).to(DEV)
    dev_ref = [o.cpu().double().numpy()
               for o in pw.fwd(*[torch.from_numpy(a).to(DEV, dtype) for a in st], t1, t2, tcx, tcy, h,
                               compute=compute)]
    host_in = [_host(a, dtype, pinned) for a in st]
    inner = lambda a: a[h:-h, h:-h, h:-h]
    for chunk in chunks:
        log("offload %s h=%d %s %s chunk %d" % ((nx, ny, nz), h, kind, mode, chunk))
        outs = [torch.full(host_in[0].shape, float("nan"), dtype=dtype, pin_memory=pinned) for _ in range(3)]
        ws = torch.empty(pw.offload_workspace_bytes(host_in[0].shape, h, dtype, chunk, compute=compute),
                         dtype=torch.uint8, device=DEV)
        with pw.tuning(copy_out=COPY_OUT[mode]):
            pw.fwd_host(*host_in, t1, t2, tcx, tcy, h, *outs, chunk, ws, compute=compute)
        torch.cuda.current_stream().synchronize()
        for q, got in enumerate(outs):
            g = got.double().numpy()
            assert within_bar(kind, inner(g), inner(ref[q]), inner(mag[q])), (chunk, q)
            assert np.array_equal(g[h:-h, h:-h], dev_ref[q][h:-h, h:-h]), (chunk, q)  # incl. zero z halo
            assert np.all(np.isnan(g[:h])) and np.all(np.isnan(g[-h:]))              # x halo planes
            assert np.all(np.isnan(g[:, :h])) and np.all(np.isnan(g[:, -h:]))        # y halo columns


@pytest.mark.parametrize("copy_out", ["kernel", "runtime", "direct", "auto"])
def test_offload_orders_on_callers_stream(pw, copy_out):
    """Work queued on the stream before the call (a device copy into the
    pinned inputs) is seen by the offload, and work queued after it (a copy
    reading the pinned outputs) sees the host results, which match the
    oracle bit for bit."""
    nx, ny, nz, seed, h = 16, 12, 64, 33, 2
    fields, _, coef = host_case(nx, ny, nz, seed)
    tzc1, tzc2, tcx, tcy = coef
    st = [oracle.pad_periodic(f, h) for f in fields]
    ref = oracle.fwd(*st, tzc1, tzc2, tcx, tcy, h)
    t1, t2 = torch.from_numpy(tzc1).to(DEV), torch.from_numpy(tzc2).to(DEV)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s), pw.tuning(copy_out=copy_out):
        dev = [torch.from_numpy(a).to(DEV, non_blocking=False) for a in st]
        host_in = [torch.empty(a.shape, dtype=torch.float64, pin_memory=True) for a in st]
        for hsrc, d in zip(host_in, dev):
            hsrc.copy_(d, non_blocking=True)                 # queued on s before the offload
        outs = [torch.zeros(host_in[0].shape, dtype=torch.float64, pin_memory=True) for _ in range(3)]
        ws = torch.empty(pw.offload_workspace_bytes(host_in[0].shape, h, torch.float64, 5), dtype=torch.uint8,
                         device=DEV)
        pw.fwd_host(*host_in, t1, t2, tcx, tcy, h, *outs, 5, ws)
        back = [torch.empty_like(o, device=DEV) for o in outs]
        for b, o in zip(back, outs):
            b.copy_(o, non_blocking=True)                    # queued on s after the offload
    s.synchronize()
    for b, r in zip(back, ref):
        bb = b.cpu().numpy()
        assert np.array_equal(bb[h:-h, h:-h, h:-h], r[h:-h, h:-h, h:-h])


def test_automatic_mode_tries_every_copy_out(pw):
    """Twelve calls in the automatic copy-out mode on the same pinned arrays:
    the first ones try each mode the outputs allow, later ones the fastest
    (and every eighth the one sampled longest ago); every call gives the bits
    of the runtime's copies."""
    nx, ny, nz, seed, h = 11, 9, 64, 37, 2
    fields, _, coef = host_case(nx, ny, nz, seed)
    tzc1, tzc2, tcx, tcy = coef
    st = [oracle.pad_periodic(f, h) for f in fields]
    t1, t2 = torch.from_numpy(tzc1).to(DEV), torch.from_numpy(tzc2).to(DEV)
    host_in = [torch.from_numpy(a).pin_memory() for a in st]
    ws = torch.empty(pw.offload_workspace_bytes(host_in[0].shape, h, torch.float64, 3), dtype=torch.uint8,
                     device=DEV)
    ref = [torch.full(host_in[0].shape, float("nan"), dtype=torch.float64, pin_memory=True) for _ in range(3)]
    with pw.tuning(copy_out="runtime"):
        pw.fwd_host(*host_in, t1, t2, tcx, tcy, h, *ref, 3, ws)
    torch.cuda.synchronize()
    for call in range(12):
        log("offload automatic call %d" % call)
        outs = [torch.full(host_in[0].shape, float("nan"), dtype=torch.float64, pin_memory=True) for _ in range(3)]
        with pw.tuning(copy_out="auto"):
            pw.fwd_host(*host_in, t1, t2, tcx, tcy, h, *outs, 3, ws)
        torch.cuda.synchronize()
        for q in range(3):
            assert np.array_equal(outs[q].numpy(), ref[q].numpy(), equal_nan=True), (call, q)


def test_offload_argument_errors(pw):
    h = 2
    shape = (8 + 2 * h, 6 + 2 * h, 64 + 2 * h)
    host = [torch.zeros(shape, dtype=torch.float64) for _ in range(6)]
    t = torch.zeros(64, dtype=torch.float64, device=DEV)
    need = pw.offload_workspace_bytes(shape, h, torch.float64, 3)
    small = torch.empty(need - 8, dtype=torch.uint8, device=DEV)
    with pytest.raises(pw.PWError) as e:
        pw.fwd_host(*host[:3], t, t, -0.005, -0.005, h, *host[3:], 3, small)
    assert e.value.code == -4
    ws = torch.empty(need, dtype=torch.uint8, device=DEV)
    with pytest.raises(pw.PWError) as e:
        pw.fwd_host(*host[:3], t, t, -0.005, -0.005, h, host[0], host[4], host[5], 3, ws)
    assert e.value.code == -2
    with pytest.raises(pw.PWError) as e:
        pw.fwd_host(*host[:3], t, t, -0.005, -0.005, h, *host[3:], 0, ws)
    assert e.value.code == -1
    # a device array in place of a host one is refused (the binding would
    # refuse it too, so call the C entry point directly)
    d = torch.zeros(shape, dtype=torch.float64, device=DEV)
    p = [pw._ptr(x) for x in host]
    rc = pw.lib.pw_advect_fwd_host(p[0], p[1], pw._ptr(d), pw._ptr(t), pw._ptr(t), -0.005, -0.005,
                                   8, 6, 64, h, p[3], p[4], p[5], 3, pw._ptr(ws), need, 0, pw._stream())
    assert rc == -1 and b"device memory" in pw.lib.pw_last_error()
