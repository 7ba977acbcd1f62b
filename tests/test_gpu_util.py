"""GPU checks of the storage utilities: device generator against the host
generator (both implement the published SplitMix64 definition), and the
periodic pad / halo kernels against the oracle's numpy padding."""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2010_01545_amd import inputs
from _helpers import H, log

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def pw():
    assert torch.cuda.is_available()
    from paper_2010_01545_amd import pwadvect
    return pwadvect


KINDS = {torch.float64: "f64", torch.float32: "f32", torch.float16: "f16", torch.bfloat16: "bf16"}


@pytest.mark.parametrize("shape", [(8, 6, 64), (5, 3, 7), (1, 1, 2)])
@pytest.mark.parametrize("dtype", list(KINDS), ids=list(KINDS.values()))
def test_fill_uniform_matches_host_generator(pw, shape, dtype):
    nx, ny, nz = shape
    log("fill %s %s" % (shape, dtype))
    for fid, amp, lids in ((inputs.FIELD_U, 10.0, False), (inputs.FIELD_W, 10.0, True),
                           (inputs.FIELD_LV, 1.0, False)):
        st = torch.full((nx + 2 * H, ny + 2 * H, nz + 2 * H), float("nan"), dtype=dtype, device=DEV)
        pw.fill_uniform(st, H, 7, fid, amp, lids)
        got = st.cpu().double().numpy()
        ref = inputs.round_storage(inputs.uniform_field(7, fid, nx, ny, nz, amp=amp, zero_lids=lids), KINDS[dtype])
        assert np.array_equal(oracle.interior(got, H), ref)
        cols = got[H:-H, H:-H]
        assert np.all(cols[:, :, :H] == 0) and np.all(cols[:, :, -H:] == 0)
        assert np.all(np.isnan(got[:H])) and np.all(np.isnan(got[:, -H:]))


@pytest.mark.parametrize("dtype", [torch.float16, torch.bfloat16], ids=["f16", "bf16"])
def test_pad_and_halo_16bit(pw, dtype):
    """The pad and halo kernels move 16-bit elements unchanged."""
    x = inputs.round_storage(np.random.default_rng(2).standard_normal((5, 4, 7)), KINDS[dtype])
    ref = oracle.pad_periodic(x, H)
    got = pw.pad_periodic(torch.from_numpy(x).to(DEV, dtype), H)
    assert np.array_equal(got.cpu().double().numpy(), ref)
    got[:H] = 3.0
    pw.halo_periodic(got, H)
    assert np.array_equal(got.cpu().double().numpy(), ref)


@pytest.mark.parametrize("shape", [(8, 6, 64), (5, 3, 7), (1, 1, 2), (2, 5, 3)])
@pytest.mark.parametrize("halo", [1, 2, 3])
def test_pad_and_halo_match_oracle(pw, shape, halo):
    nx, ny, nz = shape
    log("pad %s h=%d" % (shape, halo))
    x = np.random.default_rng(1).standard_normal(shape)
    ref = oracle.pad_periodic(x, halo)
    got = pw.pad_periodic(torch.from_numpy(x).to(DEV), halo).cpu().numpy()
    assert np.array_equal(got, ref)
    # halo fill in place from a storage array whose halos hold garbage
    st = torch.from_numpy(ref.copy()).to(DEV)
    st[:halo] = 1e300
    st[:, -halo:] = -7.0
    pw.halo_periodic(st, halo)
    assert np.array_equal(st.cpu().numpy(), ref)


@pytest.mark.parametrize("hints", [0, 1, 2, 3])
@pytest.mark.parametrize("unit,blocks", [(4, 0), (8, 0), (16, 0), (4, 7), (16, 3)])
@pytest.mark.parametrize("n", [1, 3, 6, 8])
def test_stream_copy_copies_exactly(pw, n, unit, blocks, hints):
    """The bandwidth reference copies every byte of every array, one pass or
    striding, with either cache policy on loads and stores, with a length
    that is not a multiple of a workgroup's units, and writes nothing past
    the end of its destinations."""
    log("stream copy n=%d unit=%d blocks=%d hints=%d" % (n, unit, blocks, hints))
    nbytes = 16 * 1000 + 48            # 1003 16-byte units, 4012 4-byte units
    g = torch.Generator().manual_seed(n * 100 + unit + blocks)
    src = [torch.randint(0, 255, (nbytes,), dtype=torch.uint8, generator=g).to(DEV) for _ in range(n)]
    pad = 256
    dst_full = [torch.full((nbytes + pad,), 0xA5, dtype=torch.uint8, device=DEV) for _ in range(n)]
    dst = [d[:nbytes] for d in dst_full]
    pw.stream_copy(src, dst, blocks, unit, hints)
    torch.cuda.synchronize()
    for s, d in zip(src, dst_full):
        assert torch.equal(d[:nbytes], s)
        assert torch.all(d[nbytes:] == 0xA5)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.float16])
def test_pooled_fields_give_the_same_bits(pw, dtype):
    """The forward and fused passes over arrays carved from one allocation
    (alloc_fields) give the bits they give over separately allocated arrays."""
    nx, ny, nz, h = 21, 18, 64, H
    log("pooled fields %s" % dtype)
    tzc1, tzc2, tcx, tcy = inputs.coefficients(nz)
    t1, t2 = torch.from_numpy(tzc1).to(DEV), torch.from_numpy(tzc2).to(DEV)
    shape = (nx + 2 * h, ny + 2 * h, nz + 2 * h)
    pool = pw.alloc_fields(15, shape, dtype)
    sep = [torch.empty(shape, dtype=dtype, device=DEV) for _ in range(15)]
    for arrs in (pool, sep):
        for q in range(6):
            pw.fill_uniform(arrs[q], h, 11, q, 10.0 if q < 3 else 1.0, zero_lids=(q == 2))
            pw.halo_periodic(arrs[q], h)
        for t in arrs[6:]:
            t.zero_()
        pw.fwd(*arrs[:3], t1, t2, tcx, tcy, h, *arrs[12:15])
        pw.fwd_adj(*arrs[:6], t1, t2, tcx, tcy, h, out=arrs[6:12])
    torch.cuda.synchronize()
    for a, b in zip(pool, sep):
        assert torch.equal(a, b)


def test_readme_quick_start_runs(pw):
    """The Python example of README.md runs as written, and its source terms
    match the oracle bit for bit on the interior."""
    import re
    import oracle
    from paper_2010_01545_amd import inputs
    text = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "README.md")).read()
    blocks = re.findall(r"```python\n(.*?)```", text, flags=re.S)
    assert blocks, "README.md has no python example"
    ns = {}
    exec(compile(blocks[0], "README.md", "exec"), ns)
    torch.cuda.synchronize()
    h = ns["h"]
    tzc1, tzc2, tcx, tcy = inputs.coefficients(64)
    st = [oracle.pad_periodic(a, h) for a in inputs.winds(0, 256, 256, 64)]
    ref = oracle.fwd(*st, tzc1, tzc2, tcx, tcy, h)
    for got, r in zip((ns["su"], ns["sv"], ns["sw"]), ref):
        assert np.array_equal(oracle.interior(got.cpu().numpy(), h), oracle.interior(r, h))
