"""GPU test of pw_advect_fwd_host_static, the offload entry point that
allocates nothing (its slab buffers are the library's static scratch): its
results must equal those of pw_advect_fwd_host with a caller's workspace, bit
for bit, and the FP64 oracle (bitwise for FP64, the FP32 bound for FP32), on
two calls queued back to back without a synchronisation between them, the
second on a smaller grid; a chunk whose slabs exceed the scratch is refused
before anything is queued."""
import numpy as np
import pytest
import torch

import oracle
from paper_2010_01545_amd import inputs
from _helpers import host_case, log

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def pw():
    assert torch.cuda.is_available()
    from paper_2010_01545_amd import pwadvect
    return pwadvect


def _case(nx, ny, nz, h, seed, dtype):
    fields, _, coef = host_case(nx, ny, nz, seed)
    kind = "f64" if dtype == torch.float64 else "f32"
    st = [oracle.pad_periodic(inputs.round_storage(f, kind), h) for f in fields]
    host_in = []
    for a in st:
        t = torch.empty(a.shape, dtype=dtype, pin_memory=True)
        t.copy_(torch.from_numpy(a))
        host_in.append(t)
    outs = [torch.full(host_in[0].shape, float("nan"), dtype=dtype, pin_memory=True) for _ in range(3)]
    t1, t2 = torch.from_numpy(coef[0]).to(DEV), torch.from_numpy(coef[1]).to(DEV)
    return st, coef, host_in, outs, t1, t2


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_static_scratch_matches_workspace_path_twice(pw, dtype):
    big = (512, 512, 64, 2, 41, 20)     # chunk 20: about 121 MB of the 128 MiB scratch in FP64
    small = (9, 7, 7, 2, 42, 4)
    cases = []
    for nx, ny, nz, h, seed, chunk in (big, small):
        st, coef, host_in, outs, t1, t2 = _case(nx, ny, nz, h, seed, dtype)
        need = pw.offload_workspace_bytes(host_in[0].shape, h, dtype, chunk)
        assert need <= pw.static_scratch_bytes()
        log("static offload %dx%dx%d %s chunk %d: %d scratch bytes" % (nx, ny, nz, dtype, chunk, need))
        cases.append((st, coef, host_in, outs, t1, t2, h, chunk))
    assert pw.static_scratch_bytes() == 128 << 20
    # both calls queued back to back on the current stream, the second smaller
    for st, coef, host_in, outs, t1, t2, h, chunk in cases:
        pw.fwd_host_static(*host_in, t1, t2, coef[2], coef[3], h, *outs, chunk)
    torch.cuda.current_stream().synchronize()
    for st, coef, host_in, outs, t1, t2, h, chunk in cases:
        ws = torch.empty(pw.offload_workspace_bytes(host_in[0].shape, h, dtype, chunk), dtype=torch.uint8,
                         device=DEV)
        ref_outs = [torch.full_like(o, float("nan")).pin_memory() for o in outs]
        pw.fwd_host(*host_in, t1, t2, coef[2], coef[3], h, *ref_outs, chunk, ws)
        torch.cuda.current_stream().synchronize()
        ref = oracle.fwd(*st, *coef, h)
        mag = oracle.fwd(*st, *coef, h, abs_bound=True)
        inner = lambda a: a[h:-h, h:-h, h:-h]
        for q in range(3):
            g = outs[q].double().numpy()
            r = ref_outs[q].double().numpy()
            assert np.array_equal(g[h:-h, h:-h], r[h:-h, h:-h]), q                     # same bits
            assert np.all(np.isnan(g[:h])) and np.all(np.isnan(g[:, :h]))             # halos untouched
            if dtype == torch.float64:
                assert np.array_equal(inner(g), inner(ref[q])), q
            else:
                assert not np.any(np.abs(inner(g) - inner(ref[q])) > 16 * 2.0 ** -24 * inner(mag[q])), q
        del ws


def test_static_scratch_refuses_oversized_chunk(pw):
    nx, ny, nz, h = 512, 512, 64, 2
    st, coef, host_in, outs, t1, t2 = _case(nx, ny, nz, h, 43, torch.float64)
    assert pw.offload_workspace_bytes(host_in[0].shape, h, torch.float64, 40) > pw.static_scratch_bytes()
    with pytest.raises(pw.PWError) as e:
        pw.fwd_host_static(*host_in, t1, t2, coef[2], coef[3], h, *outs, 40)
    assert e.value.code == -4
    torch.cuda.current_stream().synchronize()
    assert all(torch.isnan(o).all() for o in outs)
